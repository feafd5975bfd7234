// gfx950 kernels of libswsearch: database interleave, query profile, the
// Smith-Waterman/Gotoh sweep (16-bit packed and 32-bit cells) and top-k.
//
// Recurrence (Sec. II-B, Eq. 1-3), zero borders, S = max H:
//   H[i][j] = max(0, H[i-1][j-1] + SM(Q[i], D[j]), E[i][j], F[i][j])
//   E[i][j] = max(H[i][j-1] - Go, E[i][j-1] - Ge)
//   F[i][j] = max(H[i-1][j] - Go, F[i-1][j] - Ge)
//
// Sweep decomposition.  A wave owns P = 64/B lanes' worth of subjects of one
// length-sorted group; B lanes cooperate on each.  Lane b owns R query rows of
// every pass (a pass covers B*R consecutive rows) and, at step t, updates
// column j = t - b: the B lanes form an anti-diagonal wavefront across the
// matrix (intra-task parallelism, Sec. II-B) while the P lane groups of the
// wave are independent matrices (inter-task parallelism).  B = 1 is the pure
// inter-task sweep; B = 64 puts a whole wave on one matrix.  The bottom row of
// lane b (H and F at each column) reaches lane b+1 one step later through a
// DPP wave shift; between passes it goes through a per-wave scratch slot.
//
// The two 16-bit halves of a lane hold either two subjects of the group
// against one query (subject pairs) or one subject against two queries (query
// pairs).  Image bytes are residue code + 1, 0 for padding, so that buffer
// loads outside a group (which return zeros) read padding.
//
// Cell arithmetic.  Per cell the kernel keeps E already advanced to the next
// column and F to the next row, so H - Go is computed once and shared:
//   hd = Hdiag + SM;  H = max(hd, E, F);  S = max(S, H)
//   hgo = max(H - Go, 0);  E' = max(E - Ge, hgo);  F' = max(F - Ge, hgo)
// Flooring E and F at zero leaves every H unchanged (H >= 0 already).
// The 16-bit form keeps H, E and F plus a bias c >= -min SM (c = 4 for
// BLOSUM62), so that every value it compares, hd included, is a non-negative
// 16-bit integer; those below 0x7C00 order like the half floats with the same
// bits, while 0x7C00 and above are infinity or NaN, which v_pk_maximum3_f16
// propagates.  One maximum3 then gives H = max(hd, E, F), another E' with the
// floor c (E >= c keeps every H >= c, the local floor; F needs none), and one
// more folds two rows' H into S.  Subtractions saturate at zero
// (v_pk_sub_u16), so a value that drops below c only stands for one below
// zero, which the floors make irrelevant.  Padding rows and columns score 0:
// a padded sum is a stored value plus zero, never one of the NaN patterns
// -1023..-1, and padding cannot raise S above what the real cells reach
// (a padded cell only repeats a real value along its diagonal, and local
// cells start from the floor).  So S < kSat16 (0x7C00) is exact (no H reached
// it, so no sum was clamped) and the score is S - c; S >= kSat16 sends the
// pair to the 32-bit sweep.
#include <hip/hip_runtime.h>

#include <climits>
#include <type_traits>

#include "sw_internal.h"

namespace sw {

typedef short s2 __attribute__((ext_vector_type(2)));
typedef unsigned short u2 __attribute__((ext_vector_type(2)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

template <class To, class From>
__device__ __forceinline__ To bits(From v) { return __builtin_bit_cast(To, v); }

__device__ __forceinline__ uint32_t shr1(uint32_t v) {
    // lane l receives lane l-1's value (DPP wave_shr:1); lane 0 receives 0
    return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);
}

// ------------------------------------------------------------ buffer access
// Raw buffer resource over [base, base + bytes).  A load at an offset outside
// the range returns zeros and a store there is dropped; the sweep relies on it
// for padding columns, the zero border of a first pass and lanes with nothing
// to read or write.  Offsets are formed in the 32-bit per-lane operand, where
// a negative value wraps to a large one and is out of range too.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr uint32_t kNoAccess = 0x80000000u;   // beyond every buffer range used here (all < 2 GiB)

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    // every argument is wave-uniform; say so, or the compiler loops over lanes around each access
    const uint64_t p = (uint64_t)base;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)p), hi = __builtin_amdgcn_readfirstlane((uint32_t)(p >> 32));
    void* q = (void*)(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(q, (short)0, (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}
__device__ __forceinline__ uint32_t ld32(rsrc_t r, uint32_t off) { return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0); }
__device__ __forceinline__ uint2 ld64(rsrc_t r, uint32_t off) { return bits<uint2>(__builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0)); }
__device__ __forceinline__ uint4 ld128(rsrc_t r, uint32_t off) { return bits<uint4>(__builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0)); }
__device__ __forceinline__ void st64(rsrc_t r, uint32_t off, uint32_t x, uint32_t y) {
    __builtin_amdgcn_raw_buffer_store_b64(v2u{x, y}, r, off, 0, 0);
}
__device__ __forceinline__ void st128(rsrc_t r, uint32_t off, uint4 v) {
    __builtin_amdgcn_raw_buffer_store_b128(bits<v4u>(v), r, off, 0, 0);
}

// ------------------------------------------------------------ cell policies
// Boundary words of one column: H then F (two packed dwords in 16 bits, four
// dwords Ha, Hb, Fa, Fb in 32 bits).
struct CellI16 {
    using T = s2;
    static constexpr int kWords = 2;
    __device__ static T zero() { return T{0, 0}; }
    __device__ static T sm(uint32_t pa, uint32_t pb, int r) {
        // row r of subject a (low half) and of subject b (high half)
        return bits<T>(__builtin_amdgcn_perm(pb, pa, (r & 1) ? 0x07060302u : 0x05040100u));
    }
    __device__ static T add(T d, T s) { return __builtin_elementwise_add_sat(d, s); }
    __device__ static T gap(T x, u2 g) { return bits<T>(__builtin_elementwise_sub_sat(bits<u2>(x), g)); }
    __device__ static T mx(T a, T b) { return __builtin_elementwise_max(a, b); }
    // column u (0..3) of a 4-column boundary record
    __device__ static void col(const uint4* w, int u, T& h, T& f) {
        const uint4 v = w[u >> 1];
        h = bits<T>((u & 1) ? v.z : v.x);
        f = bits<T>((u & 1) ? v.w : v.y);
    }
    __device__ static void put(rsrc_t r, uint32_t off, T h, T f) { st64(r, off, bits<uint32_t>(h), bits<uint32_t>(f)); }
    __device__ static T shift(T v) { return bits<T>(shr1(bits<uint32_t>(v))); }
    __device__ static T sel(bool c, T a, T b) { return c ? a : b; }
    // S halves are compared as unsigned 16-bit patterns (see the header comment)
    __device__ static T xmax(T v, int mask) {
        const u2 o = bits<u2>(__shfl_xor(bits<int>(v), mask, 64));
        return bits<T>(__builtin_elementwise_max(bits<u2>(v), o));
    }
    __device__ static int lo(T v) { return (int)(unsigned short)v.x; }
    __device__ static int hi(T v) { return (int)(unsigned short)v.y; }
    using G = u2;
    __device__ static G gapv(int g) { unsigned short c = (unsigned short)(g > 65535 ? 65535 : g); return G{c, c}; }
};

struct I2 { int x, y; };

struct CellI32 {
    using T = I2;
    static constexpr int kWords = 4;
    __device__ static T zero() { return T{0, 0}; }
    __device__ static T sm(uint32_t pa, uint32_t pb, int r) {
        if (r & 1) return T{(int)pa >> 16, (int)pb >> 16};
        return T{(int)(short)(pa & 0xffffu), (int)(short)(pb & 0xffffu)};
    }
    __device__ static T add(T d, T s) { return T{d.x + s.x, d.y + s.y}; }
    __device__ static int g1(int x, unsigned g) { return (int)__builtin_elementwise_sub_sat((unsigned)x, g); }
    __device__ static T gap(T x, unsigned g) { return T{g1(x.x, g), g1(x.y, g)}; }
    __device__ static T mx(T a, T b) { return T{max(a.x, b.x), max(a.y, b.y)}; }
    __device__ static void col(const uint4* w, int u, T& h, T& f) {
        const uint4 v = w[u];
        h = T{(int)v.x, (int)v.y};
        f = T{(int)v.z, (int)v.w};
    }
    __device__ static void put(rsrc_t r, uint32_t off, T h, T f) {
        st128(r, off, make_uint4((uint32_t)h.x, (uint32_t)h.y, (uint32_t)f.x, (uint32_t)f.y));
    }
    __device__ static T shift(T v) { return T{(int)shr1((uint32_t)v.x), (int)shr1((uint32_t)v.y)}; }
    __device__ static T sel(bool c, T a, T b) { return c ? a : b; }
    __device__ static T xmax(T v, int mask) {
        return mx(v, T{__shfl_xor(v.x, mask, 64), __shfl_xor(v.y, mask, 64)});
    }
    __device__ static int lo(T v) { return v.x; }
    __device__ static int hi(T v) { return v.y; }
    using G = unsigned;
    __device__ static G gapv(int g) { return (unsigned)g; }
};

// ------------------------------------------------------------ scheduled 16-bit rows
// One column step of R rows of packed 16-bit cells, written as one asm block
// whose order never lets an instruction read the result of the packed (VOP3P)
// instruction just before it: gfx950 needs a wait state there, and the
// compiler, whose scheduler does not model that hazard, otherwise pays it with
// an s_nop on nearly every row.  Values carry the bias c (see the header
// comment), so the three-way maximum of Eq. 1 is one v_pk_maximum3_f16.  Per
// row r the block interleaves the chain H -> H-Go -> F' -> next H with
// independent work of the neighbouring rows:
//   hd'  = H[r] + SM(r+1)        next row's diagonal term, read before H[r] changes
//   H[r] = maximum3(hd, E[r], F)
//   es   = E[r] -sat Ge
//   hgo  = H[r] -sat Go
//   fs   = F -sat Ge
//   (permute of row r+2's substitution pair, subject-pair form only)
//   E[r] = maximum3(es, hgo, c)  the floor c keeps every H at c or above
//   F    = max(fs, hgo)
//   S    = maximum3(S, H[r-1], H[r])   after every odd row
// hd and hd' alternate between two registers from row to row.  This is the
// arithmetic of the generic row loop in sweep_pass, reordered and biased.
#define SWA(r, n) "v_pk_add_i16 %[d" #n "], %[h" #r "], %[sm] clamp\n"
#define SWAW(r, n, w) "v_pk_add_i16 %[d" #n "], %[h" #r "], %[w" #w "] clamp\n"
#define SWD(r, c) "v_pk_maximum3_f16 %[h" #r "], %[d" #c "], %[e" #r "], %[f]\n"
#define SWF(r) "v_pk_sub_u16 %[es], %[e" #r "], %[ge] clamp\n"
#define SWE(r) "v_pk_sub_u16 %[hgo], %[h" #r "], %[go] clamp\n"
#define SWH "v_pk_sub_u16 %[fs], %[f], %[ge] clamp\n"
#define SWP(k, sel) "v_perm_b32 %[sm], %[b" #k "], %[a" #k "], %[" #sel "]\n"
#define SWG(r) "v_pk_maximum3_f16 %[e" #r "], %[es], %[hgo], %[c]\n"
#define SWI "v_pk_max_i16 %[f], %[fs], %[hgo]\n"
#define SWM(a, b) "v_pk_maximum3_f16 %[s], %[s], %[h" #a "], %[h" #b "]\n"
// subject-pair form: row r's pair is perm(b[r/2], a[r/2]) with selector s0 (even r) or s1 (odd r);
// the prologue forms row 0's hd (register d0) and row 1's pair
#define SW_PRO "v_perm_b32 %[sm], %[b0], %[a0], %[s0]\n" "v_pk_add_i16 %[d0], %[dt], %[sm] clamp\n" SWP(0, s1)
// row r reads hd from d(r%2) and writes row r+1's into d((r+1)%2)
#define SW_BLK(r, c, n, k2, sel2) SWA(r, n) SWD(r, c) SWF(r) SWE(r) SWH SWP(k2, sel2) SWG(r) SWI
#define SW_BLKS(r, c, n, k2, sel2, rp) SW_BLK(r, c, n, k2, sel2) SWM(rp, r)
#define SW_BLKN(r, c, n) SWA(r, n) SWD(r, c) SWF(r) SWE(r) SWH SWG(r) SWI
// the last row starts with E[r] - Ge, as the block before it ends with the write of F
#define SW_LAST(r, c, rp) SWF(r) SWD(r, c) SWH SWE(r) SWM(rp, r) SWG(r) SWI
// pre-packed form: row r's pair is w[r]
#define SW_PROW "v_pk_add_i16 %[d0], %[dt], %[w0] clamp\n"
#define SW_BLKW(r, c, n, w) SWAW(r, n, w) SWD(r, c) SWF(r) SWE(r) SWH SWG(r) SWI
#define SW_BLKWS(r, c, n, w, rp) SW_BLKW(r, c, n, w) SWM(rp, r)

// End-to-end modes: no local floor (E' = max(es, hgo), one packed maximum),
// and every two rows H folds into a running maximum (%[s]) and a running
// minimum (%[lmin]) that tell whether all values stayed in the exact range.
#define SWG0(r) "v_pk_max_i16 %[e" #r "], %[es], %[hgo]\n"
#define SWN(a, b) "v_pk_minimum3_f16 %[lmin], %[lmin], %[h" #a "], %[h" #b "]\n"
#define SW_MBLK(r, c, n, k2, sel2) SWA(r, n) SWD(r, c) SWF(r) SWE(r) SWH SWP(k2, sel2) SWG0(r) SWI
#define SW_MBLKS(r, c, n, k2, sel2, rp) SW_MBLK(r, c, n, k2, sel2) SWM(rp, r) SWN(rp, r)
#define SW_MBLKN(r, c, n) SWA(r, n) SWD(r, c) SWF(r) SWE(r) SWH SWG0(r) SWI
#define SW_MLAST(r, c, rp) SWF(r) SWD(r, c) SWH SWE(r) SWM(rp, r) SWN(rp, r) SWG0(r) SWI

// Global mode on column-offset cells (H' = H - g(j), Ge <= Go): E extends for free and opens at
// Go - Ge, so E' = max(E, H' - (Go - Ge)) (%[es] holds H' - (Go - Ge), %[goe] is Go - Ge); F, the
// diagonal and the folds as above.  The last row waits one state before its maximum reads F.
#define SWX(r) "v_pk_sub_u16 %[es], %[h" #r "], %[goe] clamp\n"
#define SWG3(r) "v_pk_max_i16 %[e" #r "], %[e" #r "], %[es]\n"
#define SW_XBLK(r, c, n, k2, sel2) SWA(r, n) SWD(r, c) SWH SWX(r) SWE(r) SWP(k2, sel2) SWG3(r) SWI
#define SW_XBLKS(r, c, n, k2, sel2, rp) SW_XBLK(r, c, n, k2, sel2) SWM(rp, r) SWN(rp, r)
#define SW_XBLKN(r, c, n) SWA(r, n) SWD(r, c) SWH SWX(r) SWE(r) SWG3(r) SWI
#define SW_XLAST(r, c, rp) "s_nop 0\n" SWD(r, c) SWH SWX(r) SWE(r) SWM(rp, r) SWN(rp, r) SWG3(r) SWI

#define SW_HE(i) [h##i] "+v"(H[i]), [e##i] "+v"(E[i])
#define SW_AB(i) [a##i] "v"(pa[i]), [b##i] "v"(pb[i])
#define SW_W(i) [w##i] "v"(w[i])
#define SW_OUTS [s] "+v"(S), [f] "+v"(F), [d0] "=&v"(d0), [d1] "=&v"(d1), [hgo] "=&v"(hgo), [es] "=&v"(es), \
                [fs] "=&v"(fs)
#define SW_INS [dt] "v"(diag), [go] "s"(go), [ge] "s"(ge), [c] "s"(c)

// Subject-pair form: pa/pb hold rows 2k, 2k+1 of subject a and of subject b.
template <int R>
__device__ __forceinline__ void rows16_pair(s2* H, s2* E, s2& S, s2& F, s2 diag, const uint32_t* pa,
                                            const uint32_t* pb, u2 go, u2 ge, u2 c) {
    s2 d0, d1, hgo, es, fs, sm;
    const uint32_t s0 = 0x05040100u, s1 = 0x07060302u;
    if constexpr (R == 16) {
        asm(SW_PRO SW_BLK(0, 0, 1, 1, s0) SW_BLKS(1, 1, 0, 1, s1, 0) SW_BLK(2, 0, 1, 2, s0)
                SW_BLKS(3, 1, 0, 2, s1, 2) SW_BLK(4, 0, 1, 3, s0) SW_BLKS(5, 1, 0, 3, s1, 4) SW_BLK(6, 0, 1, 4, s0)
                    SW_BLKS(7, 1, 0, 4, s1, 6) SW_BLK(8, 0, 1, 5, s0) SW_BLKS(9, 1, 0, 5, s1, 8)
                        SW_BLK(10, 0, 1, 6, s0) SW_BLKS(11, 1, 0, 6, s1, 10) SW_BLK(12, 0, 1, 7, s0)
                            SW_BLKS(13, 1, 0, 7, s1, 12) SW_BLKN(14, 0, 1) SW_LAST(15, 1, 14)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_HE(4), SW_HE(5), SW_HE(6), SW_HE(7), SW_HE(8), SW_HE(9),
              SW_HE(10), SW_HE(11), SW_HE(12), SW_HE(13), SW_HE(14), SW_HE(15), SW_OUTS, [sm] "=&v"(sm)
            : SW_INS, SW_AB(0), SW_AB(1), SW_AB(2), SW_AB(3), SW_AB(4), SW_AB(5), SW_AB(6), SW_AB(7),
              [s0] "s"(s0), [s1] "s"(s1));
    } else if constexpr (R == 8) {
        asm(SW_PRO SW_BLK(0, 0, 1, 1, s0) SW_BLKS(1, 1, 0, 1, s1, 0) SW_BLK(2, 0, 1, 2, s0)
                SW_BLKS(3, 1, 0, 2, s1, 2) SW_BLK(4, 0, 1, 3, s0) SW_BLKS(5, 1, 0, 3, s1, 4) SW_BLKN(6, 0, 1)
                    SW_LAST(7, 1, 6)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_HE(4), SW_HE(5), SW_HE(6), SW_HE(7), SW_OUTS,
              [sm] "=&v"(sm)
            : SW_INS, SW_AB(0), SW_AB(1), SW_AB(2), SW_AB(3), [s0] "s"(s0), [s1] "s"(s1));
    } else {
        static_assert(R == 4, "rows per lane must be 4, 8 or 16");
        asm(SW_PRO SW_BLK(0, 0, 1, 1, s0) SW_BLKS(1, 1, 0, 1, s1, 0) SW_BLKN(2, 0, 1) SW_LAST(3, 1, 2)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_OUTS, [sm] "=&v"(sm)
            : SW_INS, SW_AB(0), SW_AB(1), [s0] "s"(s0), [s1] "s"(s1));
    }
}

// Pre-packed form: w[r] is row r's substitution pair.
template <int R>
__device__ __forceinline__ void rows16_packed(s2* H, s2* E, s2& S, s2& F, s2 diag, const uint32_t* w, u2 go,
                                              u2 ge, u2 c) {
    s2 d0, d1, hgo, es, fs;
    if constexpr (R == 16) {
        asm(SW_PROW SW_BLKW(0, 0, 1, 1) SW_BLKWS(1, 1, 0, 2, 0) SW_BLKW(2, 0, 1, 3) SW_BLKWS(3, 1, 0, 4, 2)
                SW_BLKW(4, 0, 1, 5) SW_BLKWS(5, 1, 0, 6, 4) SW_BLKW(6, 0, 1, 7) SW_BLKWS(7, 1, 0, 8, 6)
                    SW_BLKW(8, 0, 1, 9) SW_BLKWS(9, 1, 0, 10, 8) SW_BLKW(10, 0, 1, 11) SW_BLKWS(11, 1, 0, 12, 10)
                        SW_BLKW(12, 0, 1, 13) SW_BLKWS(13, 1, 0, 14, 12) SW_BLKW(14, 0, 1, 15) SW_LAST(15, 1, 14)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_HE(4), SW_HE(5), SW_HE(6), SW_HE(7), SW_HE(8), SW_HE(9),
              SW_HE(10), SW_HE(11), SW_HE(12), SW_HE(13), SW_HE(14), SW_HE(15), SW_OUTS
            : SW_INS, SW_W(0), SW_W(1), SW_W(2), SW_W(3), SW_W(4), SW_W(5), SW_W(6), SW_W(7), SW_W(8), SW_W(9),
              SW_W(10), SW_W(11), SW_W(12), SW_W(13), SW_W(14), SW_W(15));
    } else if constexpr (R == 8) {
        asm(SW_PROW SW_BLKW(0, 0, 1, 1) SW_BLKWS(1, 1, 0, 2, 0) SW_BLKW(2, 0, 1, 3) SW_BLKWS(3, 1, 0, 4, 2)
                SW_BLKW(4, 0, 1, 5) SW_BLKWS(5, 1, 0, 6, 4) SW_BLKW(6, 0, 1, 7) SW_LAST(7, 1, 6)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_HE(4), SW_HE(5), SW_HE(6), SW_HE(7), SW_OUTS
            : SW_INS, SW_W(0), SW_W(1), SW_W(2), SW_W(3), SW_W(4), SW_W(5), SW_W(6), SW_W(7));
    } else {
        static_assert(R == 4, "rows per lane must be 4, 8 or 16");
        asm(SW_PROW SW_BLKW(0, 0, 1, 1) SW_BLKWS(1, 1, 0, 2, 0) SW_BLKW(2, 0, 1, 3) SW_LAST(3, 1, 2)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_OUTS
            : SW_INS, SW_W(0), SW_W(1), SW_W(2), SW_W(3));
    }
}

// End-to-end modes, subject-pair form, R = 16, 8 or 4 rows: S is the running
// maximum of H, lmin the running minimum (both for the range check).
#define SW_MOUTS [s] "+v"(S), [lmin] "+v"(lmin), [f] "+v"(F), [d0] "=&v"(d0), [d1] "=&v"(d1), [hgo] "=&v"(hgo), \
                 [es] "=&v"(es), [fs] "=&v"(fs), [sm] "=&v"(sm)
#define SW_MINS [dt] "v"(diag), [go] "s"(go), [ge] "s"(ge), [s0] "s"(s0), [s1] "s"(s1)
template <int R>
__device__ __forceinline__ void rows16_pair_mode(s2* H, s2* E, s2& S, s2& lmin, s2& F, s2 diag, const uint32_t* pa,
                                                 const uint32_t* pb, u2 go, u2 ge) {
    s2 d0, d1, hgo, es, fs, sm;
    const uint32_t s0 = 0x05040100u, s1 = 0x07060302u;
    if constexpr (R == 16) {
        asm(SW_PRO SW_MBLK(0, 0, 1, 1, s0) SW_MBLKS(1, 1, 0, 1, s1, 0) SW_MBLK(2, 0, 1, 2, s0)
                SW_MBLKS(3, 1, 0, 2, s1, 2) SW_MBLK(4, 0, 1, 3, s0) SW_MBLKS(5, 1, 0, 3, s1, 4) SW_MBLK(6, 0, 1, 4, s0)
                    SW_MBLKS(7, 1, 0, 4, s1, 6) SW_MBLK(8, 0, 1, 5, s0) SW_MBLKS(9, 1, 0, 5, s1, 8)
                        SW_MBLK(10, 0, 1, 6, s0) SW_MBLKS(11, 1, 0, 6, s1, 10) SW_MBLK(12, 0, 1, 7, s0)
                            SW_MBLKS(13, 1, 0, 7, s1, 12) SW_MBLKN(14, 0, 1) SW_MLAST(15, 1, 14)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_HE(4), SW_HE(5), SW_HE(6), SW_HE(7), SW_HE(8), SW_HE(9),
              SW_HE(10), SW_HE(11), SW_HE(12), SW_HE(13), SW_HE(14), SW_HE(15), SW_MOUTS
            : SW_MINS, SW_AB(0), SW_AB(1), SW_AB(2), SW_AB(3), SW_AB(4), SW_AB(5), SW_AB(6), SW_AB(7));
    } else if constexpr (R == 8) {
        asm(SW_PRO SW_MBLK(0, 0, 1, 1, s0) SW_MBLKS(1, 1, 0, 1, s1, 0) SW_MBLK(2, 0, 1, 2, s0)
                SW_MBLKS(3, 1, 0, 2, s1, 2) SW_MBLK(4, 0, 1, 3, s0) SW_MBLKS(5, 1, 0, 3, s1, 4) SW_MBLKN(6, 0, 1)
                    SW_MLAST(7, 1, 6)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_HE(4), SW_HE(5), SW_HE(6), SW_HE(7), SW_MOUTS
            : SW_MINS, SW_AB(0), SW_AB(1), SW_AB(2), SW_AB(3));
    } else {
        static_assert(R == 4, "rows per lane must be 4, 8 or 16");
        asm(SW_PRO SW_MBLK(0, 0, 1, 1, s0) SW_MBLKS(1, 1, 0, 1, s1, 0) SW_MBLKN(2, 0, 1) SW_MLAST(3, 1, 2)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_MOUTS
            : SW_MINS, SW_AB(0), SW_AB(1));
    }
}

// Global mode on column-offset cells, subject-pair form, R = 16, 8 or 4 rows.
#define SW_XMINS [dt] "v"(diag), [go] "s"(go), [ge] "s"(ge), [goe] "s"(goe), [s0] "s"(s0), [s1] "s"(s1)
template <int R>
__device__ __forceinline__ void rows16_pair_xmode(s2* H, s2* E, s2& S, s2& lmin, s2& F, s2 diag, const uint32_t* pa,
                                                  const uint32_t* pb, u2 go, u2 ge, u2 goe) {
    s2 d0, d1, hgo, es, fs, sm;
    const uint32_t s0 = 0x05040100u, s1 = 0x07060302u;
    if constexpr (R == 16) {
        asm(SW_PRO SW_XBLK(0, 0, 1, 1, s0) SW_XBLKS(1, 1, 0, 1, s1, 0) SW_XBLK(2, 0, 1, 2, s0)
                SW_XBLKS(3, 1, 0, 2, s1, 2) SW_XBLK(4, 0, 1, 3, s0) SW_XBLKS(5, 1, 0, 3, s1, 4) SW_XBLK(6, 0, 1, 4, s0)
                    SW_XBLKS(7, 1, 0, 4, s1, 6) SW_XBLK(8, 0, 1, 5, s0) SW_XBLKS(9, 1, 0, 5, s1, 8)
                        SW_XBLK(10, 0, 1, 6, s0) SW_XBLKS(11, 1, 0, 6, s1, 10) SW_XBLK(12, 0, 1, 7, s0)
                            SW_XBLKS(13, 1, 0, 7, s1, 12) SW_XBLKN(14, 0, 1) SW_XLAST(15, 1, 14)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_HE(4), SW_HE(5), SW_HE(6), SW_HE(7), SW_HE(8), SW_HE(9),
              SW_HE(10), SW_HE(11), SW_HE(12), SW_HE(13), SW_HE(14), SW_HE(15), SW_MOUTS
            : SW_XMINS, SW_AB(0), SW_AB(1), SW_AB(2), SW_AB(3), SW_AB(4), SW_AB(5), SW_AB(6), SW_AB(7));
    } else if constexpr (R == 8) {
        asm(SW_PRO SW_XBLK(0, 0, 1, 1, s0) SW_XBLKS(1, 1, 0, 1, s1, 0) SW_XBLK(2, 0, 1, 2, s0)
                SW_XBLKS(3, 1, 0, 2, s1, 2) SW_XBLK(4, 0, 1, 3, s0) SW_XBLKS(5, 1, 0, 3, s1, 4) SW_XBLKN(6, 0, 1)
                    SW_XLAST(7, 1, 6)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_HE(4), SW_HE(5), SW_HE(6), SW_HE(7), SW_MOUTS
            : SW_XMINS, SW_AB(0), SW_AB(1), SW_AB(2), SW_AB(3));
    } else {
        static_assert(R == 4, "rows per lane must be 4, 8 or 16");
        asm(SW_PRO SW_XBLK(0, 0, 1, 1, s0) SW_XBLKS(1, 1, 0, 1, s1, 0) SW_XBLKN(2, 0, 1) SW_XLAST(3, 1, 2)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_MOUTS
            : SW_XMINS, SW_AB(0), SW_AB(1));
    }
}

// ------------------------------------------------------------ one pass of one wave
// Where a pass reads and writes.  The image resource covers the group's chunk
// rows; the boundary resource covers the wave's slot for this unit, laid out
// [chunk][lane group][4 columns][kWords], exactly nchunks chunks long, so that
// columns at or past the unit's width read as zero and are never written.
struct PassIO {
    rsrc_t img;
    uint32_t img_lane;     // byte offset of this lane's residues within a chunk row
    rsrc_t bnd;
    uint32_t rd_lane;      // byte offset of this lane group's boundary words in a chunk, or kNoAccess
    uint32_t wr_lane;      // same for the writing lane, or kNoAccess
    uint32_t cstride;      // boundary bytes per chunk (all lane groups)
};

// Residues of 4 columns: two subjects (x: a, y: b) or one.
template <bool PACKED> struct Res;
template <> struct Res<false> {
    using V = uint2;
    __device__ static V load(rsrc_t r, uint32_t off) { return ld64(r, off); }
    __device__ static V align(V hi, V lo, int sh) {
        return make_uint2(__builtin_amdgcn_alignbyte(hi.x, lo.x, sh), __builtin_amdgcn_alignbyte(hi.y, lo.y, sh));
    }
};
template <> struct Res<true> {
    using V = uint32_t;
    __device__ static V load(rsrc_t r, uint32_t off) { return ld32(r, off); }
    __device__ static V align(V hi, V lo, int sh) { return __builtin_amdgcn_alignbyte(hi, lo, sh); }
};

// Profile values of one step (R dwords): subject pairs read R int16 of each
// subject ([residue][R] int16 slice), query pairs read R dwords of their one
// residue ([residue][R] dword slice, halves already interleaved).
template <int R, bool PACKED>
__device__ __forceinline__ void fetch(const int16_t* lrow, typename Res<PACKED>::V rr, int u, uint32_t* out) {
    if constexpr (PACKED) {
        const int d = (rr >> (8 * u)) & 0xff;
        const uint4* q = reinterpret_cast<const uint4*>(reinterpret_cast<const uint32_t*>(lrow) + d * R);
#pragma unroll
        for (int v = 0; v < R / 4; ++v) {
            const uint4 x = q[v];
            out[4 * v] = x.x; out[4 * v + 1] = x.y; out[4 * v + 2] = x.z; out[4 * v + 3] = x.w;
        }
    } else {
        const int da = (rr.x >> (8 * u)) & 0xff;
        const int db = (rr.y >> (8 * u)) & 0xff;
        if constexpr (R % 8 == 0) {
            const uint4* qa = reinterpret_cast<const uint4*>(lrow + da * R);
            const uint4* qb = reinterpret_cast<const uint4*>(lrow + db * R);
#pragma unroll
            for (int v = 0; v < R / 8; ++v) {
                const uint4 x = qa[v], y = qb[v];
                out[4 * v] = x.x; out[4 * v + 1] = x.y; out[4 * v + 2] = x.z; out[4 * v + 3] = x.w;
                out[R / 2 + 4 * v] = y.x; out[R / 2 + 4 * v + 1] = y.y;
                out[R / 2 + 4 * v + 2] = y.z; out[R / 2 + 4 * v + 3] = y.w;
            }
        } else {
            static_assert(R == 4, "rows per lane must be 4 or a multiple of 8");
            const uint2 x = *reinterpret_cast<const uint2*>(lrow + da * R);
            const uint2 y = *reinterpret_cast<const uint2*>(lrow + db * R);
            out[0] = x.x; out[1] = x.y; out[2] = y.x; out[3] = y.y;
        }
    }
}

// Rows [p*B*R, (p+1)*B*R) of the query (or of both queries) against columns
// [0, ncols) of the lane's matrices.  `lrow` points at this lane's profile
// rows in LDS.  H, E, F live in registers; the boundary row between passes
// goes through the slot.  Profile values of the next step are read from LDS
// while the current step computes; residues are read two chunks ahead.
// Global and semi-global modes (32-bit cells only): no local floor, gap-run
// borders g(k) = -(Go + (k-1) min(Go, Ge)) on column 0 (and on row 0 for
// global; 0 for semi-global), S taken on the query's last row: at the
// subject's last column (global) or its best column (semi-global).
struct EndCtx {
    int row0;                 // 0-based first query row of this lane in this pass
    int m;                    // query length
    int na, nb;               // lengths of the lane's two subjects
    int go, ge, ext;          // Go, Ge, min(Go, Ge)
    bool top;                 // pass 0: row 0 is the border
    bool last;                // the last pass: it holds the query's last row
    int bias;                 // 16-bit cells: the bias every value carries
    int smshift;              // 32-bit cells: subtracted from every profile value (the profile of column-offset
                              // global cells carries SM + smshift)
    __device__ int border(int k) const { return k <= 0 ? 0 : -(go + (k - 1) * ext); }
    // a value as a biased 16-bit cell, clamped to [0, 0x7FFF] (a clamped value fails the range check)
    __device__ short enc(int v) const { v += bias; return (short)(v < 0 ? 0 : v > 0x7FFF ? 0x7FFF : v); }
};

template <class C, int R, bool COOP, bool PACKED, int MODE = 0>
__device__ __forceinline__ void sweep_pass(const PassIO& io, int ncols, int B, int b, const int16_t* lrow,
                                           typename C::G go, typename C::G ge, typename C::T& S, typename C::T bias,
                                           const EndCtx& ec = EndCtx{}) {
    static_assert(MODE == 0 || std::is_same<C, CellI32>::value, "end-to-end modes use 32-bit cells");
    using T = typename C::T;
    using RV = typename Res<PACKED>::V;
    constexpr int W = C::kWords;
    const int nsteps = ncols + B - 1;
    const int nloop = (nsteps + 3) >> 2;
    const bool first_lane = (b == 0);

    T H[R], E[R];      // H and E of this lane's rows at the last column done (biased, 16-bit cells)
#pragma unroll
    for (int r = 0; r < R; ++r) { H[r] = bias; E[r] = bias; }
    T diag = bias;               // H of the row above this lane's block, previous column
    T up_h = C::zero(), up_f = C::zero();   // bottom row of lane b-1, one column back
    if constexpr (MODE != 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int hb = ec.border(ec.row0 + r + 1);               // H[i][0]
            H[r] = T{hb, hb};
            E[r] = T{hb - ec.go, hb - ec.go};                         // E[i][1]: E[i][0] is minus infinity
        }
        const int hb = ec.border(ec.row0);                            // H[row above][0]
        diag = T{hb, hb};
        up_h = T{hb, hb};             // what lane b-1 hands over before its first column: its last row's border
    }
    const int rcap = ec.m - 1 - ec.row0;    // row of this lane holding the query's last row, if in 0..R-1

    // lane b works on columns 4c - b .. 4c - b + 3 during iteration c
    const int coff = COOP ? ((-b) >> 2) : 0;      // floor((-b)/4)
    const int csh = COOP ? ((-b) & 3) : 0;
    auto res_at = [&](int c) { return Res<PACKED>::load(io.img, io.img_lane + (uint32_t)(c * kChunkBytes)); };
    auto resid = [&](RV lo, RV hi) { return COOP ? Res<PACKED>::align(hi, lo, csh) : lo; };
    RV c0 = res_at(coff), c1 = res_at(coff + 1), c2 = res_at(coff + 2);

    uint4 bw[W];                 // boundary words of the current 4 columns (first lane of a pass > 0)
#pragma unroll
    for (int i = 0; i < W; ++i) bw[i] = ld128(io.bnd, io.rd_lane + 16u * i);

    RV rr = resid(c0, c1);
    // Profile values are read from LDS two steps before the step that uses them (cur: this step,
    // nxt: the next), so each read has a whole step of cell updates to complete in, whatever waits the
    // compiler places; a lone wave (a long subject's chain) would otherwise stall on LDS every few steps.
    // 32-bit cells and query pairs keep one step of lead (the registers of a second one would lower
    // their occupancy).
    constexpr bool kLead2 = std::is_same<C, CellI16>::value && !PACKED;
    uint32_t cur[R], nxt[R];
    fetch<R, PACKED>(lrow, rr, 0, cur);
    if constexpr (kLead2) fetch<R, PACKED>(lrow, rr, 1, nxt);
    for (int c = 0; c < nloop; ++c) {
        const RV c3 = res_at(coff + c + 3);
        uint4 nw[W];
#pragma unroll
        for (int i = 0; i < W; ++i) nw[i] = ld128(io.bnd, io.rd_lane + (uint32_t)(c + 1) * io.cstride + 16u * i);
        const RV rn = resid(c1, c2);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            uint32_t nx2[R];
            if constexpr (kLead2) {
                if (u < 2) fetch<R, PACKED>(lrow, rr, u + 2, nx2);
                else fetch<R, PACKED>(lrow, rn, u - 2, nx2);
            } else {
                if (u < 3) fetch<R, PACKED>(lrow, rr, u + 1, nxt);
                else fetch<R, PACKED>(lrow, rn, 0, nxt);
            }
            T htop, ftop;
            C::col(bw, u, htop, ftop);
            if (COOP) {
                htop = C::sel(first_lane, htop, up_h);
                ftop = C::sel(first_lane, ftop, up_f);
            }
            // the zero border of a first pass reads as zeros: raise it to the bias (F may stay below it)
            if constexpr (std::is_same<C, CellI16>::value) htop = C::mx(htop, bias);
            const int col = 4 * c + u - (COOP ? b : 0);               // 0-based column of this step
            if constexpr (MODE != 0) {
                if (first_lane && ec.top) {                           // row 0 of the matrix
                    const int h0 = MODE == 1 ? ec.border(col + 1) : 0;
                    htop = T{h0, h0};
                    ftop = T{h0 - ec.go, h0 - ec.go};
                }
            }
            T F = ftop;
            if constexpr (MODE != 0) {
                auto rows = [&]() {
                    T dg = diag;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const T sv = C::sm(cur[r >> 1], cur[R / 2 + (r >> 1)], r);
                        const T hd = T{dg.x + sv.x - ec.smshift, dg.y + sv.y - ec.smshift};
                        const T h = T{max(max(hd.x, E[r].x), F.x), max(max(hd.y, E[r].y), F.y)};
                        dg = H[r];
                        H[r] = h;
                        E[r] = T{max(E[r].x - ec.ge, h.x - ec.go), max(E[r].y - ec.ge, h.y - ec.go)};
                        F = T{max(F.x - ec.ge, h.x - ec.go), max(F.y - ec.ge, h.y - ec.go)};
                        if (ec.last && r == rcap) {
                            if (MODE == 1) {
                                if (col == ec.na - 1) S.x = h.x;
                                if (col == ec.nb - 1) S.y = h.y;
                            } else {
                                if (col < ec.na) S.x = max(S.x, h.x);
                                if (col < ec.nb) S.y = max(S.y, h.y);
                            }
                        }
                    }
                };
                // a cooperating lane starts b steps late and keeps the border until its first column;
                // once the wave's last lane has started (a wave-uniform test) no lane needs the guard
                if (!COOP || 4 * c + u >= B - 1) rows();
                else if (col >= 0) rows();
            } else if constexpr (std::is_same<C, CellI16>::value) {
                if constexpr (PACKED) rows16_packed<R>(H, E, S, F, diag, cur, go, ge, bits<u2>(bias));
                else rows16_pair<R>(H, E, S, F, diag, cur, cur + R / 2, go, ge, bits<u2>(bias));
            } else {
                T dg = diag;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    T hd = C::add(dg, C::sm(cur[r >> 1], cur[R / 2 + (r >> 1)], r));
                    T h = C::mx(C::mx(hd, E[r]), F);
                    S = C::mx(S, h);
                    dg = H[r];
                    H[r] = h;
                    T hgo = C::gap(h, go);
                    E[r] = C::mx(C::gap(E[r], ge), hgo);
                    F = C::mx(C::gap(F, ge), hgo);
                }
            }
            diag = htop;
            const T hbot = H[R - 1];
            // the last lane of a lane group hands column j = t - (B - 1) to the next pass
            const int j = 4 * c + u - (B - 1);
            C::put(io.bnd, io.wr_lane + (uint32_t)((j >> 2) * (int)io.cstride + (j & 3) * 4 * W), hbot, F);
            if (COOP) {
                up_h = C::shift(hbot);
                up_f = C::shift(F);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cur[r] = nxt[r];
                if constexpr (kLead2) nxt[r] = nx2[r];
            }
        }
        c0 = c1;
        c1 = c2;
        c2 = c3;
        rr = rn;
#pragma unroll
        for (int i = 0; i < W; ++i) bw[i] = nw[i];
    }
}

// End-to-end modes in 16-bit cells (subject pairs, R rows per lane).  Values
// carry the bias ec.bias (the middle of the 16-bit range for plain global
// cells, just above -g(m) for semi-global and column-offset global cells, which
// hold H - g(j) and never fall below g(m)), so that
// H = max(hd, E, F) is one v_pk_maximum3_f16 as in the local sweep; there is
// no floor, and a subtraction that saturates at 0 only stands for a value
// below the range.  lmin and lmax fold every H: while all of a pair's H stay
// in [kModeLo, a.sat) (and its borders are representable), every value is
// exact; otherwise the pair is recomputed in 32-bit cells.  Padding scores 0,
// so padded cells copy real values diagonally rather than leaving the range,
// and the borders of padded rows and columns repeat the last real ones.
constexpr int kModeLo = 128;       // lowest safe biased H: H + SM stays >= 0 for every int8 SM

__device__ __forceinline__ short usub16(short v, int g) {
    const int x = (int)(unsigned short)v - g;
    return (short)(x < 0 ? 0 : x);
}

template <int R, bool COOP, int MODE>
__device__ __forceinline__ void sweep_pass_mode16(const PassIO& io, int ncols, int B, int b, const int16_t* lrow,
                                                  u2 go, u2 ge, s2& S, s2& lmin, s2& lmax, const EndCtx& ec) {
    using C = CellI16;
    using T = s2;
    using RV = Res<false>::V;
    constexpr int W = C::kWords;
    const int nsteps = ncols + B - 1;
    const int nloop = (nsteps + 3) >> 2;
    const bool first_lane = (b == 0);

    // Column-offset global cells: column 0 is not offset, but as the diagonal of column 1 it reads
    // g(i) + Go - Ge (the diagonal into column 1 gains Go, of which the profile adds Ge), and
    // E'[i][1] = E[i][1] - g(1) = g(i).
    constexpr bool kOff = MODE == kModeGlobalOffset;
    const int dshift = kOff ? ec.go - ec.ext : 0;
    const u2 goe = C::gapv(ec.go - ec.ext);
    T H[R], E[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int hv = ec.border(min(ec.row0 + r + 1, ec.m));              // H[i][0]; padded rows repeat row m's
        const short hb = ec.enc(hv + dshift);
        H[r] = T{hb, hb};
        const short e = kOff ? ec.enc(hv) : usub16(hb, ec.go);              // E[i][1]
        E[r] = T{e, e};
    }
    const short hb0 = ec.enc(ec.border(min(ec.row0, ec.m)) + dshift);
    T diag = T{hb0, hb0};          // H[row above][0]
    T up_h = diag, up_f = C::zero();   // what lane b-1 hands over before its first column
    const int rcap = ec.m - 1 - ec.row0;
    const bool cap = ec.last && rcap >= 0 && rcap < R;     // this lane holds the query's last row

    const int coff = COOP ? ((-b) >> 2) : 0;
    const int csh = COOP ? ((-b) & 3) : 0;
    auto res_at = [&](int c) { return Res<false>::load(io.img, io.img_lane + (uint32_t)(c * kChunkBytes)); };
    auto resid = [&](RV lo, RV hi) { return COOP ? Res<false>::align(hi, lo, csh) : lo; };
    RV c0 = res_at(coff), c1 = res_at(coff + 1), c2 = res_at(coff + 2);
    uint4 bw[W];
#pragma unroll
    for (int i = 0; i < W; ++i) bw[i] = ld128(io.bnd, io.rd_lane + 16u * i);
    RV rr = resid(c0, c1);
    uint32_t cur[R];
    fetch<R, false>(lrow, rr, 0, cur);
    for (int c = 0; c < nloop; ++c) {
        const RV c3 = res_at(coff + c + 3);
        uint4 nw[W];
#pragma unroll
        for (int i = 0; i < W; ++i) nw[i] = ld128(io.bnd, io.rd_lane + (uint32_t)(c + 1) * io.cstride + 16u * i);
        const RV rn = resid(c1, c2);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            uint32_t nxt[R];
            if (u < 3) fetch<R, false>(lrow, rr, u + 1, nxt);
            else fetch<R, false>(lrow, rn, 0, nxt);
            T htop, ftop;
            C::col(bw, u, htop, ftop);
            if (COOP) {
                htop = C::sel(first_lane, htop, up_h);
                ftop = C::sel(first_lane, ftop, up_f);
            }
            const int col = 4 * c + u - (COOP ? b : 0);
            if (first_lane && ec.top) {
                // row 0: the gap-run border (plain global cells; padded columns repeat the last real one), or
                // 0 (semi-global, and column-offset global cells, where it is g(j) - g(j))
                const short ta = ec.enc(MODE == 1 ? ec.border(min(col + 1, ec.na)) : 0);
                const short tb = ec.enc(MODE == 1 ? ec.border(min(col + 1, ec.nb)) : 0);
                htop = T{ta, tb};
                ftop = T{usub16(ta, ec.go), usub16(tb, ec.go)};
            }
            T F = ftop;
            // a cooperating lane starts b steps late and keeps the border until its first column (the
            // asm block runs under the lane mask)
            if (!COOP || col >= 0) {
                if constexpr (kOff) rows16_pair_xmode<R>(H, E, lmax, lmin, F, diag, cur, cur + R / 2, go, ge, goe);
                else rows16_pair_mode<R>(H, E, lmax, lmin, F, diag, cur, cur + R / 2, go, ge);
            }
            if (cap) {
                T hc = H[0];
#pragma unroll
                for (int r = 1; r < R; ++r)
                    if (r == rcap) hc = H[r];
                if (col >= 0) {                     // a lane before its first column captures nothing
                    if (MODE == 1 || kOff) {
                        if (col == ec.na - 1) S.x = hc.x;
                        if (col == ec.nb - 1) S.y = hc.y;
                    } else {
                        if (col < ec.na) S.x = max(S.x, hc.x);
                        if (col < ec.nb) S.y = max(S.y, hc.y);
                    }
                }
            }
            diag = htop;
            const T hbot = H[R - 1];
            const int j = 4 * c + u - (B - 1);
            C::put(io.bnd, io.wr_lane + (uint32_t)((j >> 2) * (int)io.cstride + (j & 3) * 4 * W), hbot, F);
            if (COOP) {
                up_h = C::shift(hbot);
                up_f = C::shift(F);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) cur[r] = nxt[r];
        }
        c0 = c1;
        c1 = c2;
        c2 = c3;
        rr = rn;
#pragma unroll
        for (int i = 0; i < W; ++i) bw[i] = nw[i];
    }
}

// Load rows [row0, row0 + B*R) of a query profile into LDS as [b][residue][R],
// in 16-byte units (8-byte units when R = 4).
template <int R>
__device__ __forceinline__ void load_slice(int16_t* dst, const int16_t* prof, int mp, int row0, int lgB,
                                           int tid, int nthreads) {
    constexpr int U = (R % 8 == 0) ? 8 : 4;            // int16 elements per copy unit
    using V = typename std::conditional<U == 8, uint4, uint2>::type;
    const int rows = R << lgB;
    const int per_res = rows / U;                      // units per residue row
    const int total = kNRes * per_res;
    for (int e = tid; e < total; e += nthreads) {
        const int d = e / per_res;
        const int rem = e - d * per_res;               // = b * (R/U) + ru
        const int bb = rem / (R / U);
        const int ru = rem - bb * (R / U);
        const V v = *reinterpret_cast<const V*>(prof + (int64_t)d * mp + row0 + rem * U);
        *reinterpret_cast<V*>(dst + (bb * kNRes + d) * R + ru * U) = v;
    }
}

// Rows [row0, row0 + B*R) of two query profiles interleaved into LDS as
// [b][residue][R] dwords (low half query a, high half query b).  Rows past a
// profile's stride read as padding.
template <int R>
__device__ __forceinline__ void load_slice_q2(uint32_t* dst, const int16_t* pa, int mpa, const int16_t* pb, int mpb,
                                              int row0, int lgB, int tid, int nthreads) {
    const int rows = R << lgB;
    const int per_res = rows / 8;                       // 8-row units per residue
    const int total = kNRes * per_res;
    for (int e = tid; e < total; e += nthreads) {
        const int d = e / per_res;
        const int rem = e - d * per_res;
        const int row = row0 + rem * 8;
        const int bb = (rem * 8) / R;
        const int r0 = rem * 8 - bb * R;
        constexpr uint32_t kPad2 = (uint32_t)(uint16_t)kPadScore * 0x10001u;
        uint4 va = make_uint4(kPad2, kPad2, kPad2, kPad2), vb = va;
        if (row < mpa) va = *reinterpret_cast<const uint4*>(pa + (int64_t)d * mpa + row);
        if (row < mpb) vb = *reinterpret_cast<const uint4*>(pb + (int64_t)d * mpb + row);
        uint4 o0, o1;
        o0.x = __builtin_amdgcn_perm(vb.x, va.x, 0x05040100u); o0.y = __builtin_amdgcn_perm(vb.x, va.x, 0x07060302u);
        o0.z = __builtin_amdgcn_perm(vb.y, va.y, 0x05040100u); o0.w = __builtin_amdgcn_perm(vb.y, va.y, 0x07060302u);
        o1.x = __builtin_amdgcn_perm(vb.z, va.z, 0x05040100u); o1.y = __builtin_amdgcn_perm(vb.z, va.z, 0x07060302u);
        o1.z = __builtin_amdgcn_perm(vb.w, va.w, 0x05040100u); o1.w = __builtin_amdgcn_perm(vb.w, va.w, 0x07060302u);
        uint4* o = reinterpret_cast<uint4*>(dst + (bb * kNRes + d) * R + r0);
        o[0] = o0;
        o[1] = o1;
    }
}

// A flagged (query, subject pair) goes to the list while it has room and to
// its bit in rerun_bits after that, so that none is lost however many
// saturate; the recompute reads both.
__device__ __forceinline__ void append_rerun(const SweepArgs& a, int g, int q, int pair) {
    const int idx = atomicAdd(a.rerun_count, 1);
    if (idx < a.rerun_cap) a.rerun[idx] = WgItem{g, q, (int16_t)pair, 6, 1, 1};
    else atomicOr(a.rerun_bits + ((int64_t)q * a.rerun_groups + g) * 2 + (pair >> 5), 1u << (pair & 31));
}

// One unit of a wave: lane groups [k*P, (k+1)*P) of group g, all passes.
// Subject pairs (PACKED = false): P = 64/B pairs, one query.  Query pairs
// (PACKED = true): P = 64/B subjects, queries qpairs[q].x and .y.
template <class C, int R, bool PACKED, int MODE = 0>
__device__ __forceinline__ void run_unit(const SweepArgs& a, int g, int k, int lgB, int q, bool valid,
                                         bool shared_slice, int16_t* lds, int wave, int lane, uint32_t* slot) {
    using T = typename C::T;
    const int B = 1 << lgB;
    const int P = kGroupPairs >> lgB;
    const int s = lane >> lgB;
    const int b = lane & (B - 1);
    int qa = q, qb = -1;
    if constexpr (PACKED) {
        const int2 pr = a.qpairs[q];
        qa = pr.x;
        qb = pr.y;
    }
    const QDesc Qa = a.qd[qa];
    const QDesc Qb = a.qd[qb >= 0 ? qb : qa];
    const int m = max(Qa.m, Qb.m);
    const int rows_pp = R << lgB;
    const int passes = (m + rows_pp - 1) / rows_pp;
    const int su = k * P + s;                   // pair (subject pairs) or subject (query pairs) in the group
    GroupRec G{0, 0, 0};
    int ncols = 0;
    if (valid) {
        G = a.groups[g];
        // pairs are sorted by length within the group: the unit's first one is its widest
        ncols = a.pair_cols[g * kGroupPairs + (PACKED ? (k * P) >> 1 : k * P)];
    }
    PassIO io;
    io.img = make_rsrc(a.image + G.base, (uint32_t)(G.ncols >> 2) * kChunkBytes);
    io.img_lane = PACKED ? (uint32_t)((su >> 1) * 8 + (su & 1) * 4) : (uint32_t)(su * 8);
    io.cstride = (uint32_t)(P * 16 * C::kWords);
    io.bnd = make_rsrc(slot, (uint32_t)(ncols >> 2) * io.cstride);
    const uint32_t lane_words = (uint32_t)(s * 16 * C::kWords);
    uint32_t* region32 = reinterpret_cast<uint32_t*>(shared_slice ? lds : lds + wave * (kNRes * 16 * R));
    const int16_t* lrow = PACKED ? reinterpret_cast<const int16_t*>(region32 + b * kNRes * R)
                                 : reinterpret_cast<const int16_t*>(region32) + b * kNRes * R;
    const typename C::G go = C::gapv(a.go), ge = C::gapv(a.ge);
    T bias = C::zero();
    int ub = 0;                                 // subtracted from every score on the way out
    if constexpr (std::is_same<C, CellI16>::value) {
        bias = bits<T>((uint32_t)(uint16_t)a.bias * 0x10001u);
        ub = a.bias;
    }
    T S = bias;
    constexpr bool kMode16 = MODE != 0 && std::is_same<C, CellI16>::value;
    T lmin = C::zero(), lmax = C::zero();       // 16-bit end-to-end modes: range of every H
    EndCtx ec{};
    if constexpr (MODE != 0) {
        ec.m = m;
        ec.go = a.go;
        ec.ge = a.ge;
        ec.ext = min(a.go, a.ge);
        ec.smshift = a.sm_shift;
        const int slot0 = g * kGroupSubjects + 2 * su;
        ec.na = valid ? a.slen[slot0] : 0;
        ec.nb = valid ? a.slen[slot0 + 1] : 0;
        // the lane holding the query's last row starts S at H[m][0] where that counts
        const bool cap = (m - 1 - (passes - 1) * rows_pp) / R == b;
        if constexpr (kMode16) {
            ec.bias = a.bias;
            const short hm = ec.enc(ec.border(m));
            S = T{cap && (MODE == 2 || ec.na == 0) ? hm : (short)0, cap && (MODE == 2 || ec.nb == 0) ? hm : (short)0};
            // the extreme borders (column 0 at the last row; row 0 at the last column, global) must fit too
            const short ta = MODE == 1 ? ec.enc(ec.border(ec.na)) : hm, tb = MODE == 1 ? ec.enc(ec.border(ec.nb)) : hm;
            lmin = T{min(hm, ta), min(hm, tb)};
        } else {
            constexpr int kNeg = -(1 << 30);
            const int hm = ec.border(m);
            S = T{cap && (MODE == 2 || ec.na == 0) ? hm : kNeg, cap && (MODE == 2 || ec.nb == 0) ? hm : kNeg};
        }
    }
    // A unit with many lanes per matrix is a long subject: its passes are one
    // serial chain of steps that can outlast the rest of the search, so its
    // wave issues ahead of the other waves of its SIMD while it runs.
    const bool chain = lgB >= 5;
    if (chain) __builtin_amdgcn_s_setprio(2);
    for (int p = 0; p < passes; ++p) {
        if (shared_slice) {
            __syncthreads();
            if constexpr (PACKED)
                load_slice_q2<R>(region32, a.prof + Qa.prof_off, Qa.mp, a.prof + Qb.prof_off, Qb.mp, p * rows_pp, lgB,
                                 threadIdx.x, blockDim.x);
            else
                load_slice<R>(reinterpret_cast<int16_t*>(region32), a.prof + Qa.prof_off, Qa.mp, p * rows_pp, lgB,
                              threadIdx.x, blockDim.x);
            __syncthreads();
        } else {
            __builtin_amdgcn_wave_barrier();
            if constexpr (PACKED)
                load_slice_q2<R>(region32, a.prof + Qa.prof_off, Qa.mp, a.prof + Qb.prof_off, Qb.mp, p * rows_pp, lgB,
                                 lane, 64);
            else
                load_slice<R>(reinterpret_cast<int16_t*>(region32), a.prof + Qa.prof_off, Qa.mp, p * rows_pp, lgB,
                              lane, 64);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
        if (valid) {
            io.rd_lane = (b == 0 && p > 0) ? lane_words : kNoAccess;
            io.wr_lane = (b == B - 1 && p + 1 < passes) ? lane_words : kNoAccess;
            ec.row0 = p * rows_pp + b * R;
            ec.top = p == 0;
            ec.last = p == passes - 1;
            if constexpr (kMode16) {
                if (lgB == 0)
                    sweep_pass_mode16<R, false, MODE>(io, ncols, B, b, lrow, go, ge, S, lmin, lmax, ec);
                else
                    sweep_pass_mode16<R, true, MODE>(io, ncols, B, b, lrow, go, ge, S, lmin, lmax, ec);
            } else {
                if (lgB == 0)
                    sweep_pass<C, R, false, PACKED, MODE>(io, ncols, B, b, lrow, go, ge, S, bias, ec);
                else
                    sweep_pass<C, R, true, PACKED, MODE>(io, ncols, B, b, lrow, go, ge, S, bias, ec);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");   // boundary stores visible to the next pass
    }
    if (chain) __builtin_amdgcn_s_setprio(0);
    if (!valid) return;
    for (int o = 1; o < B; o <<= 1) S = C::xmax(S, o);
    int out_of_range = 0;                       // 16-bit end-to-end: some value left the exact range
    if constexpr (kMode16) {
        const bool ra = (unsigned short)lmin.x < kModeLo || (unsigned short)lmax.x >= (unsigned)a.sat;
        const bool rb = (unsigned short)lmin.y < kModeLo || (unsigned short)lmax.y >= (unsigned)a.sat;
        out_of_range = (ra || rb) ? 1 : 0;
        for (int o = 1; o < B; o <<= 1) out_of_range |= __shfl_xor(out_of_range, o, 64);
    }
    if constexpr (PACKED) {
        // The recompute takes subject pairs: subjects su and su ^ 1 (lane groups s and s ^ 1, B lanes
        // apart, in the same unit since P >= 2) share one flag per query, and only the even one appends it.
        int fa = a.rerun != nullptr && C::lo(S) >= a.sat;
        int fb = a.rerun != nullptr && qb >= 0 && C::hi(S) >= a.sat;
        fa |= __shfl_xor(fa, B, 64);
        fb |= __shfl_xor(fb, B, 64);
        if (b != 0) return;
        const int o = a.perm[g * kGroupSubjects + su];
        if (o >= 0) {
            int32_t* outa = Qa.out ? Qa.out : a.scores + Qa.out_off;
            outa[o] = a.poison && fa ? kPoison : C::lo(S) - ub;
            if (qb >= 0) {
                int32_t* outb = Qb.out ? Qb.out : a.scores + Qb.out_off;
                outb[o] = a.poison && fb ? kPoison : C::hi(S) - ub;
            }
        }
        if ((su & 1) == 0) {
            if (fa) append_rerun(a, g, qa, su >> 1);
            if (fb) append_rerun(a, g, qb, su >> 1);
        }
    } else {
        if (b != 0) return;
        bool flag = false;                      // the pair must be recomputed with 32-bit cells
        if (a.rerun != nullptr) flag = kMode16 ? out_of_range != 0 : (C::lo(S) >= a.sat || C::hi(S) >= a.sat);
        const bool poisoned = flag && a.poison;
        const int slot0 = g * kGroupSubjects + 2 * su;
        const int o0 = a.perm[slot0], o1 = a.perm[slot0 + 1];
        int32_t* out = Qa.out ? Qa.out : a.scores + Qa.out_off;
        // column-offset global cells hold H'[m][n] = H[m][n] - g(n)
        const int ra = MODE == kModeGlobalOffset ? ec.border(ec.na) : 0;
        const int rb = MODE == kModeGlobalOffset ? ec.border(ec.nb) : 0;
        if (o0 >= 0) out[o0] = poisoned ? kPoison : C::lo(S) - ub + ra;
        if (o1 >= 0) out[o1] = poisoned ? kPoison : C::hi(S) - ub + rb;
        if (flag) append_rerun(a, g, qa, su);
    }
}

// Recompute items past the list: blocks of kBitsBlock words of the flag bits.
constexpr int kBitsBlock = 64;

template <class C, int R, int MODE = 0>
__global__ __launch_bounds__(64 * kWaves) void k_sweep(SweepArgs a) {
    // one shared slice of up to 64*R rows, or four per-wave slices of up to 16*R rows
    __shared__ __attribute__((aligned(16))) int16_t lds[kNRes * 64 * R];
    __shared__ int s_item;
    __shared__ uint32_t s_bits[kBitsBlock];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: buffer resources stay scalar
    const int lane = threadIdx.x & 63;
    uint32_t* slot = a.scratch + ((int64_t)(a.slot_base + blockIdx.x) * kWaves + wave) * a.slot_words;
    int n_items = a.n_items, n_list = a.n_items;
    if (a.n_items_dev) {
        // recompute: the flagged pairs are the list's first min(count, capacity) entries, then (when the
        // list overflowed) every set bit of rerun_bits, read kBitsBlock words per item
        const int c = *a.n_items_dev;
        n_list = min(c, a.n_items);
        n_items = n_list;
        if (c > a.n_items) n_items += (int)((a.rerun_words + kBitsBlock - 1) / kBitsBlock);
    }
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (it >= n_items) break;
        if constexpr (std::is_same<C, CellI32>::value) {
            if (a.unit_list) {
                // 32-bit recompute, one unit per workgroup computed by wave 0 with the whole LDS slice: a
                // listed pair, or every pair whose flag bit is set in a block of kBitsBlock words (all
                // threads read the same words from LDS, so the workgroup runs the same units and barriers)
                const bool listed = it < n_list;
                WgItem I{};
                int64_t w0 = 0;
                if (listed) I = a.items[it];
                else {
                    w0 = (int64_t)(it - n_list) * kBitsBlock;
                    if (threadIdx.x < kBitsBlock) {
                        const int64_t w = w0 + threadIdx.x;
                        s_bits[threadIdx.x] = w < a.rerun_words ? a.rerun_bits[w] : 0u;
                    }
                    __syncthreads();
                }
                int done = 0, wi = 0;
                uint32_t v = 0;
                for (;;) {
                    int g, k, q;
                    if (listed) {
                        if (done) break;
                        g = I.g0;
                        k = I.k0;
                        q = I.q;
                    } else {
                        while (v == 0 && wi < kBitsBlock) v = s_bits[wi++];
                        if (v == 0) break;
                        const int bit = __builtin_ctz(v);
                        v &= v - 1;
                        const int64_t w = w0 + wi - 1;
                        q = (int)(w / (2 * (int64_t)a.rerun_groups));
                        const int rem = (int)(w - (int64_t)q * 2 * a.rerun_groups);
                        g = rem >> 1;
                        k = ((rem & 1) << 5) + bit;
                    }
                    run_unit<C, R, false, MODE>(a, g, k, 6, q, wave == 0, true, lds, wave, lane, slot);
                    ++done;
                }
                if (threadIdx.x == 0 && done) atomicAdd(a.recomputed, done);
                continue;
            }
        }
        const WgItem I = a.items[it];
        {
            const int B = 1 << I.lgB;
            int k = I.k0 + wave;
            const int g = I.g0 + (k >> I.lgB) * I.gstep;
            k &= B - 1;
            const bool shared_slice = I.lgB > 4;        // more than 16 lanes per pair
            run_unit<C, R, false, MODE>(a, g, k, I.lgB, I.q, wave < I.count, shared_slice, lds, wave, lane, slot);
        }
    }
}

// ------------------------------------------------------------ query-pair sweep
// Two queries per lane: the two halves of every packed cell are the same
// subject against query a and query b, so a row's substitution pair is one
// dword of a pre-interleaved profile slice and needs no permute.  A wave owns
// P = 64/B subjects of a group (B lanes each, anti-diagonal as above); a group
// has 2B such units.
template <int R>
__global__ __launch_bounds__(64 * kWaves) void k_sweep_q2(SweepArgs a) {
    __shared__ __attribute__((aligned(16))) int16_t lds[kNRes * 64 * R];
    __shared__ int s_item;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: buffer resources stay scalar
    const int lane = threadIdx.x & 63;
    uint32_t* slot = a.scratch + ((int64_t)(a.slot_base + blockIdx.x) * kWaves + wave) * a.slot_words;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (it >= a.n_items) break;
        const WgItem I = a.items[it];
        const int units = 2 << I.lgB;                   // units per group
        int k = I.k0 + wave;
        const int g = I.g0 + (k / units) * I.gstep;
        k %= units;
        const bool shared_slice = I.lgB > 3;            // more than 8 lanes per subject
        run_unit<CellI16, R, true>(a, g, k, I.lgB, I.q, wave < I.count, shared_slice, lds, wave, lane, slot);
    }
}

// ------------------------------------------------------------ query profile
// prof[d][i] = SM(Q[i], d - 1) + add for image codes d = 1..A and i < m
// (add = Ge for column-offset global cells, else 0); kPadScore for d = 0
// (padding), d > A and past m.  One staging buffer holds the A x A
// matrix (in a kMaxAlphabet^2-byte region) followed by the query codes.
// Thread 0 also zeroes the launch counters (they are consumed by later kernels
// on the same stream).
// The blocks of query 0 also clear the recompute's flag bits.
__global__ void k_profile(const int8_t* stage, int A, const QDesc* qd, int nq, const int64_t* qoff,
                          int16_t* prof, int32_t* counters, int ncounters, uint32_t* bits, int64_t nbits_words,
                          int add) {
    const int q = blockIdx.y;
    if (q == 0 && blockIdx.x == 0 && threadIdx.x < ncounters) counters[threadIdx.x] = 0;
    if (q == 0)
        for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nbits_words; w += (int64_t)gridDim.x * blockDim.x)
            bits[w] = 0;
    if (q >= nq) return;
    const QDesc Q = qd[q];
    const int8_t* sm = stage;
    const int8_t* query = stage + kMaxAlphabet * kMaxAlphabet + qoff[q];
    const int64_t total = (int64_t)kNRes * Q.mp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int d = (int)(e / Q.mp);
        const int i = (int)(e - (int64_t)d * Q.mp);
        int16_t v = kPadScore;
        if (d >= 1 && d <= A && i < Q.m) v = (int16_t)(sm[query[i] * A + (d - 1)] + add);
        prof[Q.prof_off + e] = v;
    }
}

// ------------------------------------------------------------ database interleave
// One thread per output dword: 4 consecutive columns of one subject.
__global__ void k_interleave(const int8_t* res, const int64_t* soff, const int32_t* slen, int64_t n, int A,
                             const GroupRec* groups, const int64_t* gdw, int ngroups, uint32_t* image,
                             int64_t total_dw, int32_t* err) {
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < total_dw; w += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = ngroups - 1;        // last group with gdw[g] <= w
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (gdw[mid] <= w) lo = mid; else hi = mid - 1;
        }
        const int g = lo;
        const int64_t local = w - gdw[g];
        const int64_t c = local / (kChunkBytes / 4);
        const int rem = (int)(local - c * (kChunkBytes / 4));    // 0..127 = 2*pair + half
        const int64_t sidx = (int64_t)g * kGroupSubjects + rem;
        uint32_t word = 0;                   // padding
        if (sidx < n) {
            const int64_t off = soff[sidx];
            const int len = slen[sidx];
            for (int kk = 0; kk < 4; ++kk) {
                const int64_t col = 4 * c + kk;
                uint32_t v = kPadCode;
                if (col < len) {
                    const int r = res[off + col];
                    if (r < 0 || r >= A) atomicOr(err, 1);
                    else v = (uint32_t)r + 1;
                }
                word |= v << (8 * kk);
            }
        }
        image[w] = word;
    }
}

// ------------------------------------------------------------ top-k
// One workgroup of 1024 threads per score row.  Radix select finds the k-th
// largest score T; every score > T and the first (k - #>T) scores equal to T in
// index order are gathered, then sorted by (score desc, index asc) with a
// bitonic network in LDS.  Positions past the row length hold (-1, -1).
constexpr int kTopkThreads = 1024;

__device__ __forceinline__ bool key_before(int sa, int64_t ia, int sb, int64_t ib) {
    return sa > sb || (sa == sb && ia < ib);
}

// Long rows go in two launches: the row is cut into nchunks pieces whose own
// top k (sorted) land side by side in a candidate row, then one workgroup takes
// the top k of the candidates.  Equal scores keep index order across the
// candidate row (pieces are in index order and each piece's list is sorted by
// index among equal scores), so the second launch's positional tie rule is
// the index rule; idx_map turns its positions back into subject indices.
__global__ __launch_bounds__(kTopkThreads) void k_topk(const int32_t* scores, int64_t n_all, int64_t row_stride, int k,
                                                       int32_t* top_s, int64_t* top_i, int nchunks, int64_t chunk_len,
                                                       const int64_t* idx_map) {
    __shared__ int hist[256];
    __shared__ int s_digit, s_rank;
    __shared__ int c_gt, c_eq;
    __shared__ int wave_cnt[kTopkThreads / 64];
    __shared__ int cand_s[1024];
    __shared__ int64_t cand_i[1024];
    const int tid = threadIdx.x;
    const int rw = blockIdx.x / nchunks, piece = blockIdx.x - rw * nchunks;
    const int64_t base = (int64_t)piece * chunk_len;
    const int64_t n = max<int64_t>(0, min<int64_t>(chunk_len, n_all - base));
    const int32_t* row = scores + (int64_t)rw * row_stride + base;
    const int64_t* imap = idx_map ? idx_map + (int64_t)rw * row_stride + base : nullptr;
    int32_t* outs = top_s + (int64_t)blockIdx.x * k;
    int64_t* outi = top_i + (int64_t)blockIdx.x * k;
    const int take = (int)min<int64_t>((int64_t)k, n);

    // radix select on the scores with the sign bit flipped (signed order as unsigned)
    uint32_t prefix = 0, mask = 0;
    int rank = take;                 // rank of the threshold among scores matching the prefix
    const bool select = take > 0 && take < n;   // else every score qualifies
    if (select) {
        for (int shift = 24; shift >= 0; shift -= 8) {
            for (int i = tid; i < 256; i += kTopkThreads) hist[i] = 0;
            __syncthreads();
            for (int64_t i = tid; i < n; i += kTopkThreads) {
                const uint32_t v = (uint32_t)row[i] ^ 0x80000000u;
                if ((v & mask) == prefix) atomicAdd(&hist[(v >> shift) & 255], 1);
            }
            __syncthreads();
            if (tid == 0) {
                int cum = 0, d = 255;
                for (; d > 0; --d) {
                    if (cum + hist[d] >= rank) break;
                    cum += hist[d];
                }
                s_digit = d;
                s_rank = rank - cum;
            }
            __syncthreads();
            prefix |= (uint32_t)s_digit << shift;
            mask |= 255u << shift;
            rank = s_rank;
            __syncthreads();
        }
    }
    const int T = (int)(prefix ^ 0x80000000u);                 // the k-th largest score
    const int need_eq = select ? rank : 0;
    if (tid == 0) { c_gt = 0; c_eq = 0; }
    __syncthreads();
    for (int64_t base = 0; base < n && take > 0; base += kTopkThreads) {
        const int64_t i = base + tid;
        const bool in = i < n;
        const int v = in ? row[i] : 0;
        const bool gt = in && (!select || v > T);
        const bool eq = in && select && v == T;
        if (gt) {
            const int pos = atomicAdd(&c_gt, 1);
            if (pos < take) { cand_s[pos] = v; cand_i[pos] = i; }
        }
        const uint64_t bal = __ballot(eq);
        const int w = tid >> 6, l = tid & 63;
        const int before = __popcll(bal & ((1ull << l) - 1ull));
        if (l == 0) wave_cnt[w] = __popcll(bal);
        __syncthreads();
        int off = c_eq;
        for (int x = 0; x < w; ++x) off += wave_cnt[x];
        if (eq) {
            const int pos = off + before;
            if (pos < need_eq) { cand_s[take - need_eq + pos] = v; cand_i[take - need_eq + pos] = i; }
        }
        __syncthreads();
        if (tid == 0) {
            int tot = 0;
            for (int x = 0; x < kTopkThreads / 64; ++x) tot += wave_cnt[x];
            c_eq += tot;
        }
        __syncthreads();
    }
    // bitonic sort of cand[0, take) padded to a power of two
    int sz = 1;
    while (sz < take) sz <<= 1;
    for (int i = tid; i < sz; i += kTopkThreads)
        if (i >= take) { cand_s[i] = INT_MIN; cand_i[i] = INT64_MAX; }
    __syncthreads();
    for (int len = 2; len <= sz; len <<= 1) {
        for (int st = len >> 1; st > 0; st >>= 1) {
            for (int i = tid; i < sz; i += kTopkThreads) {
                const int jx = i ^ st;
                if (jx > i) {
                    const bool asc = (i & len) == 0;      // "ascending" = best first in this block
                    const bool swap = asc ? key_before(cand_s[jx], cand_i[jx], cand_s[i], cand_i[i])
                                          : key_before(cand_s[i], cand_i[i], cand_s[jx], cand_i[jx]);
                    if (swap) {
                        const int ts = cand_s[i]; cand_s[i] = cand_s[jx]; cand_s[jx] = ts;
                        const int64_t ti = cand_i[i]; cand_i[i] = cand_i[jx]; cand_i[jx] = ti;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < k; i += kTopkThreads) {
        if (i < take) { outs[i] = cand_s[i]; outi[i] = imap ? imap[cand_i[i]] : base + cand_i[i]; }
        else { outs[i] = -1; outi[i] = -1; }
    }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ------------------------------------------------------------ host-side launchers
// Kernel instances: 16-bit cells with R = 4, 8, 16 rows per lane; 32-bit cells with R = 8.
static const void* sweep_kernel_q2(int R) {
    if (R == 8) return (const void*)k_sweep_q2<8>;
    if (R == 16) return (const void*)k_sweep_q2<16>;
    return nullptr;
}

hipError_t launch_sweep_q2(int R, const SweepArgs& a, int grid, hipStream_t st) {
    const void* k = sweep_kernel_q2(R);
    if (!k) return hipErrorInvalidValue;
    SweepArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(k, dim3(grid), dim3(64 * kWaves), args, 0, st);
}

hipError_t sweep_occupancy_q2(int R, int* blocks_per_cu) {
    const void* k = sweep_kernel_q2(R);
    if (!k) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, 64 * kWaves, 0);
}

static const void* sweep_kernel(bool i16, int R) {
    if (i16) {
        if (R == 4) return (const void*)k_sweep<CellI16, 4>;
        if (R == 8) return (const void*)k_sweep<CellI16, 8>;
        if (R == 16) return (const void*)k_sweep<CellI16, 16>;
        return nullptr;
    }
    if (R == 8) return (const void*)k_sweep<CellI32, 8>;
    return nullptr;
}

hipError_t launch_sweep(bool i16, int R, const SweepArgs& a, int grid, hipStream_t st) {
    const void* k = sweep_kernel(i16, R);
    if (!k) return hipErrorInvalidValue;
    SweepArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(k, dim3(grid), dim3(64 * kWaves), args, 0, st);
}

// Global (mode 1) and semi-global (mode 2) sweeps: 32-bit cells, R = 8.
static const void* mode_kernel(int mode, int R) {
    if (R != 8) return nullptr;
    if (mode == 1) return (const void*)k_sweep<CellI32, 8, 1>;
    if (mode == 2) return (const void*)k_sweep<CellI32, 8, 2>;
    return nullptr;
}

static const void* mode16_kernel(int mode, int R) {
    if (mode == 1)
        return R == 16 ? (const void*)k_sweep<CellI16, 16, 1>
             : R == 8  ? (const void*)k_sweep<CellI16, 8, 1>
             : R == 4  ? (const void*)k_sweep<CellI16, 4, 1> : nullptr;
    if (mode == 2)
        return R == 16 ? (const void*)k_sweep<CellI16, 16, 2>
             : R == 8  ? (const void*)k_sweep<CellI16, 8, 2>
             : R == 4  ? (const void*)k_sweep<CellI16, 4, 2> : nullptr;
    if (mode == 3)
        return R == 16 ? (const void*)k_sweep<CellI16, 16, 3>
             : R == 8  ? (const void*)k_sweep<CellI16, 8, 3>
             : R == 4  ? (const void*)k_sweep<CellI16, 4, 3> : nullptr;
    return nullptr;
}

// End-to-end modes in 16-bit cells (R = 16, 8 or 4 rows per lane); out-of-range pairs go to the rerun list.
hipError_t launch_sweep_mode16(int mode, int R, const SweepArgs& a, int grid, hipStream_t st) {
    const void* k = mode16_kernel(mode, R);
    if (!k) return hipErrorInvalidValue;
    SweepArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(k, dim3(grid), dim3(64 * kWaves), args, 0, st);
}

hipError_t sweep_occupancy_mode16(int mode, int R, int* blocks_per_cu) {
    const void* k = mode16_kernel(mode, R);
    if (!k) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, 64 * kWaves, 0);
}

// End-to-end modes in 32-bit cells (8 rows per lane).
hipError_t launch_sweep_mode(int mode, int R, const SweepArgs& a, int grid, hipStream_t st) {
    const void* k = mode_kernel(mode, R);
    if (!k) return hipErrorInvalidValue;
    SweepArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(k, dim3(grid), dim3(64 * kWaves), args, 0, st);
}


hipError_t sweep_occupancy(bool i16, int R, int* blocks_per_cu) {
    const void* k = sweep_kernel(i16, R);
    if (!k) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, 64 * kWaves, 0);
}

hipError_t launch_profile(const int8_t* stage, int A, const QDesc* qd, int nq, const int64_t* qoff, int16_t* prof,
                          int32_t* counters, int ncounters, uint32_t* bits, int64_t nbits_words, int max_mp,
                          hipStream_t st, int add) {
    const int64_t work = std::max<int64_t>((int64_t)kNRes * max_mp, nbits_words);
    const int bx = (int)std::min<int64_t>((work + 255) / 256, 1024);
    hipLaunchKernelGGL(k_profile, dim3(bx, std::max(nq, 1)), dim3(256), 0, st, stage, A, qd, nq, qoff, prof,
                       counters, ncounters, bits, nbits_words, add);
    return hipGetLastError();
}

hipError_t launch_interleave(const int8_t* res, const int64_t* soff, const int32_t* slen, int64_t n, int A,
                             const GroupRec* groups, const int64_t* gdw, int ngroups, uint32_t* image,
                             int64_t total_dw, int32_t* err, hipStream_t st) {
    const int64_t blocks = std::min<int64_t>((total_dw + 255) / 256, 65536);
    hipLaunchKernelGGL(k_interleave, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, res, soff, slen, n,
                       A, groups, gdw, ngroups, image, total_dw, err);
    return hipGetLastError();
}

hipError_t launch_topk(const int32_t* scores, int64_t n, int64_t row_stride, int rows, int k, int32_t* top_s,
                       int64_t* top_i, hipStream_t st) {
    hipLaunchKernelGGL(k_topk, dim3(rows), dim3(kTopkThreads), 0, st, scores, n, row_stride, k, top_s, top_i, 1, n,
                       nullptr);
    return hipGetLastError();
}

// Pieces for the two-launch top-k of rows x n scores (1 = one launch).
// Pieces of about 4,096 scores: one workgroup per piece keeps the first launch
// spread over many CUs (a 570,000-score row takes 140), and the merge sorts
// pieces x k candidates.
int topk_pieces(int64_t n, int rows, int k) {
    if (n < (int64_t)4 * kTopkThreads * 4 || rows >= 128) return 1;
    int64_t p = (n + 4095) / 4096;
    p = std::min<int64_t>(p, std::max(1, 256 / std::max(rows, 1)));
    return (int)std::max<int64_t>(p, 1);
}

int64_t topk_ws_bytes(int64_t n, int rows, int k) {
    const int p = topk_pieces(n, rows, k);
    if (p <= 1) return 0;
    return (int64_t)rows * p * k * (int64_t)(sizeof(int32_t) + sizeof(int64_t)) + 256;
}

hipError_t launch_topk_ws(const int32_t* scores, int64_t n, int64_t row_stride, int rows, int k, int32_t* top_s,
                          int64_t* top_i, void* ws, hipStream_t st) {
    const int p = topk_pieces(n, rows, k);
    if (p <= 1 || !ws) return launch_topk(scores, n, row_stride, rows, k, top_s, top_i, st);
    const int64_t cand = (int64_t)p * k;                     // candidates per row
    int64_t* ci = static_cast<int64_t*>(ws);
    int32_t* cs = reinterpret_cast<int32_t*>(ci + (int64_t)rows * cand);
    const int64_t chunk = (n + p - 1) / p;
    hipLaunchKernelGGL(k_topk, dim3(rows * p), dim3(kTopkThreads), 0, st, scores, n, row_stride, k, cs, ci, p, chunk,
                       nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_topk, dim3(rows), dim3(kTopkThreads), 0, st, cs, cand, cand, k, top_s, top_i, 1, cand,
                       (const int64_t*)ci);
    return hipGetLastError();
}

hipError_t launch_fill(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace sw
