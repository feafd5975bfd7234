// gfx950 kernels of libswsearch: database interleave, query profile, the
// Smith-Waterman/Gotoh sweep (16-bit packed and 32-bit cells) and top-k.
//
// Recurrence (Sec. II-B, Eq. 1-3), zero borders, S = max H:
//   H[i][j] = max(0, H[i-1][j-1] + SM(Q[i], D[j]), E[i][j], F[i][j])
//   E[i][j] = max(H[i][j-1] - Go, E[i][j-1] - Ge)
//   F[i][j] = max(H[i-1][j] - Go, F[i-1][j] - Ge)
//
// Sweep decomposition.  A wave owns P = 64/B subject pairs of one length-sorted
// group; B lanes cooperate on each pair.  Lane b of a pair owns R query rows
// of every pass (a pass covers B*R consecutive rows) and, at step t, updates
// column j = t - b of both subjects of its pair: the B lanes form an
// anti-diagonal wavefront across the matrix (intra-task parallelism, Sec. II-B)
// while the P pairs of the wave are independent matrices (inter-task
// parallelism).  B = 1 is the pure inter-task sweep; B = 64 puts a whole wave
// on one pair.  The bottom row of lane b (H and F at each column) reaches
// lane b+1 one step later through a DPP wave shift; between passes it goes
// through a per-wave scratch slot in global memory.
//
// Cell arithmetic.  Per cell the kernel keeps E already advanced to the next
// column and F to the next row, so H - Go is computed once and shared:
//   hd = Hdiag + SM;  H = max(hd, E, F);  S = max(S, hd)
//   hgo = max(H - Go, 0);  E' = max(E - Ge, hgo);  F' = max(F - Ge, hgo)
// Flooring E and F at zero leaves every H unchanged (H >= 0 already), and
// S = max(S, hd) equals max(S, H) because E and F never exceed an earlier H.
// The 16-bit form packs the two subjects of a pair into one VGPR and uses
// saturating v_pk_add_i16 / v_pk_sub_u16 / v_pk_max_i16: a clamped sum forces
// the cell, hence S, to 32767, so any S < 32767 is exact and S = 32767 sends
// the pair to the 32-bit sweep.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sw_internal.h"

namespace sw {

typedef short s2 __attribute__((ext_vector_type(2)));
typedef unsigned short u2 __attribute__((ext_vector_type(2)));

template <class To, class From>
__device__ __forceinline__ To bits(From v) { return __builtin_bit_cast(To, v); }

__device__ __forceinline__ uint32_t shr1(uint32_t v) {
    // lane l receives lane l-1's value, lane 0 receives 0 (DPP wave_shr:1)
    return __builtin_amdgcn_update_dpp(0u, v, 0x138, 0xf, 0xf, false);
}

// ------------------------------------------------------------ cell policies
struct CellI16 {
    using T = s2;
    static constexpr int kWords = 2;           // boundary words per (column, pair): H, F
    __device__ static T zero() { return T{0, 0}; }
    __device__ static T sm(uint32_t pa, uint32_t pb, int r) {
        // row r of subject a (low half) and of subject b (high half)
        return bits<T>(__builtin_amdgcn_perm(pb, pa, (r & 1) ? 0x07060302u : 0x05040100u));
    }
    __device__ static T add(T d, T s) { return __builtin_elementwise_add_sat(d, s); }
    __device__ static T gap(T x, u2 g) { return bits<T>(__builtin_elementwise_sub_sat(bits<u2>(x), g)); }
    __device__ static T mx(T a, T b) { return __builtin_elementwise_max(a, b); }
    __device__ static void put(uint32_t* w, T h, T f) { *reinterpret_cast<uint2*>(w) = make_uint2(bits<uint32_t>(h), bits<uint32_t>(f)); }
    __device__ static T shift(T v) { return bits<T>(shr1(bits<uint32_t>(v))); }
    __device__ static T sel(bool c, T a, T b) { return c ? a : b; }
    __device__ static T xmax(T v, int mask) {
        return mx(v, bits<T>(__shfl_xor(bits<int>(v), mask, 64)));
    }
    __device__ static int lo(T v) { return v.x; }
    __device__ static int hi(T v) { return v.y; }
    using G = u2;
    __device__ static G gapv(int g) { unsigned short c = (unsigned short)(g > 65535 ? 65535 : g); return G{c, c}; }
};

struct I2 { int x, y; };

struct CellI32 {
    using T = I2;
    static constexpr int kWords = 4;           // Ha, Hb, Fa, Fb
    __device__ static T zero() { return T{0, 0}; }
    __device__ static T sm(uint32_t pa, uint32_t pb, int r) {
        if (r & 1) return T{(int)pa >> 16, (int)pb >> 16};
        return T{(int)(short)(pa & 0xffffu), (int)(short)(pb & 0xffffu)};
    }
    __device__ static T add(T d, T s) { return T{d.x + s.x, d.y + s.y}; }
    __device__ static int g1(int x, unsigned g) { return (int)__builtin_elementwise_sub_sat((unsigned)x, g); }
    __device__ static T gap(T x, unsigned g) { return T{g1(x.x, g), g1(x.y, g)}; }
    __device__ static T mx(T a, T b) { return T{max(a.x, b.x), max(a.y, b.y)}; }
    __device__ static void put(uint32_t* w, T h, T f) {
        *reinterpret_cast<uint4*>(w) = make_uint4((uint32_t)h.x, (uint32_t)h.y, (uint32_t)f.x, (uint32_t)f.y);
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

template <class C>
__device__ __forceinline__ void ld_words(const uint32_t* p, typename C::T& h, typename C::T& f);
template <>
__device__ __forceinline__ void ld_words<CellI16>(const uint32_t* p, s2& h, s2& f) {
    uint2 v = *reinterpret_cast<const uint2*>(p);
    h = bits<s2>(v.x);
    f = bits<s2>(v.y);
}
template <>
__device__ __forceinline__ void ld_words<CellI32>(const uint32_t* p, I2& h, I2& f) {
    uint4 v = *reinterpret_cast<const uint4*>(p);
    h = I2{(int)v.x, (int)v.y};
    f = I2{(int)v.z, (int)v.w};
}

__device__ __forceinline__ uint2 load_chunk(const uint8_t* resp, int c, int nchunks) {
    if (c < 0 || c >= nchunks) return make_uint2(0x14141414u, 0x14141414u);
    return *reinterpret_cast<const uint2*>(resp + (int64_t)c * kChunkBytes);
}

// ------------------------------------------------------------ scheduled 16-bit rows
// One column step of R rows of packed 16-bit cells, written as one asm block
// whose order never lets an instruction read the result of the packed (VOP3P)
// instruction just before it: gfx950 needs a wait state there, and the
// compiler, whose scheduler does not model that hazard, otherwise pays it with
// an s_nop on nearly every row.  Per row r the block interleaves the chain
// H -> H-Go -> F' -> next H with independent work of the neighbouring rows:
//   hd   = H[r] + SM(r+1)        next row's diagonal term, read before H[r] changes
//   H[r] = max(t, F)             t = max(hd_r, E[r]) from the row before
//   es   = E[r] -sat Ge
//   hgo  = H[r] -sat Go
//   fs   = F -sat Ge
//   (permute of row r+2's substitution pair, subject-pair form only)
//   t    = max(hd, E[r+1])
//   E[r] = max(es, hgo)
//   F    = max(fs, hgo)
//   S    = max(S, hd)
// This is the arithmetic of the generic row loop in sweep_pass, reordered.
#define SWA(r) "v_pk_add_i16 %[hd], %[h" #r "], %[sm] clamp\n"
#define SWAW(r, n) "v_pk_add_i16 %[hd], %[h" #r "], %[w" #n "] clamp\n"
#define SWD(r) "v_pk_max_i16 %[h" #r "], %[t], %[f]\n"
#define SWF(r) "v_pk_sub_u16 %[es], %[e" #r "], %[ge] clamp\n"
#define SWE(r) "v_pk_sub_u16 %[hgo], %[h" #r "], %[go] clamp\n"
#define SWH "v_pk_sub_u16 %[fs], %[f], %[ge] clamp\n"
#define SWP(k, sel) "v_perm_b32 %[sm], %[b" #k "], %[a" #k "], %[" #sel "]\n"
#define SWB(n) "v_pk_max_i16 %[t], %[hd], %[e" #n "]\n"
#define SWG(r) "v_pk_max_i16 %[e" #r "], %[es], %[hgo]\n"
#define SWI "v_pk_max_i16 %[f], %[fs], %[hgo]\n"
#define SWC "v_pk_max_i16 %[s], %[s], %[hd]\n"
// subject-pair form: row r's pair is perm(b[r/2], a[r/2]) with selector s0 (even r) or s1 (odd r)
#define SW_PRO "v_perm_b32 %[sm], %[b0], %[a0], %[s0]\n" "v_pk_add_i16 %[hd], %[dt], %[sm] clamp\n" SWP(0, s1) SWB(0) SWC
#define SW_BLK(r, n, k2, sel2) SWA(r) SWD(r) SWF(r) SWE(r) SWH SWP(k2, sel2) SWB(n) SWG(r) SWI SWC
#define SW_BLKN(r, n) SWA(r) SWD(r) SWF(r) SWE(r) SWH SWB(n) SWG(r) SWI SWC
#define SW_LAST(r) SWD(r) SWF(r) SWE(r) SWH SWG(r) SWI
// pre-packed form: row r's pair is w[r]; the prologue takes row 0's F - Ge
#define SW_PROW "v_pk_add_i16 %[hd], %[dt], %[w0] clamp\n" SWH SWB(0) SWC
#define SW_BLK0W SWAW(0, 1) SWD(0) SWF(0) SWE(0) SWB(1) SWG(0) SWI SWC
#define SW_BLKW(r, n) SWAW(r, n) SWD(r) SWF(r) SWE(r) SWH SWB(n) SWG(r) SWI SWC

#define SW_HE(i) [h##i] "+v"(H[i]), [e##i] "+v"(E[i])
#define SW_AB(i) [a##i] "v"(pa[i]), [b##i] "v"(pb[i])
#define SW_W(i) [w##i] "v"(w[i])
#define SW_OUTS [s] "+v"(S), [f] "+v"(F), [hd] "=&v"(hd), [t] "=&v"(t), [hgo] "=&v"(hgo), [es] "=&v"(es), \
                [fs] "=&v"(fs)
#define SW_INS [dt] "v"(diag), [go] "s"(go), [ge] "s"(ge)

// Subject-pair form: pa/pb hold rows 2k, 2k+1 of subject a and of subject b.
template <int R>
__device__ __forceinline__ void rows16_pair(s2* H, s2* E, s2& S, s2& F, s2 diag, const uint32_t* pa,
                                            const uint32_t* pb, u2 go, u2 ge) {
    s2 hd, t, hgo, es, fs, sm;
    const uint32_t s0 = 0x05040100u, s1 = 0x07060302u;
    if constexpr (R == 16) {
        asm(SW_PRO SW_BLK(0, 1, 1, s0) SW_BLK(1, 2, 1, s1) SW_BLK(2, 3, 2, s0) SW_BLK(3, 4, 2, s1)
                SW_BLK(4, 5, 3, s0) SW_BLK(5, 6, 3, s1) SW_BLK(6, 7, 4, s0) SW_BLK(7, 8, 4, s1)
                    SW_BLK(8, 9, 5, s0) SW_BLK(9, 10, 5, s1) SW_BLK(10, 11, 6, s0) SW_BLK(11, 12, 6, s1)
                        SW_BLK(12, 13, 7, s0) SW_BLK(13, 14, 7, s1) SW_BLKN(14, 15) SW_LAST(15)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_HE(4), SW_HE(5), SW_HE(6), SW_HE(7), SW_HE(8), SW_HE(9),
              SW_HE(10), SW_HE(11), SW_HE(12), SW_HE(13), SW_HE(14), SW_HE(15), SW_OUTS, [sm] "=&v"(sm)
            : SW_INS, SW_AB(0), SW_AB(1), SW_AB(2), SW_AB(3), SW_AB(4), SW_AB(5), SW_AB(6), SW_AB(7),
              [s0] "s"(s0), [s1] "s"(s1));
    } else if constexpr (R == 8) {
        asm(SW_PRO SW_BLK(0, 1, 1, s0) SW_BLK(1, 2, 1, s1) SW_BLK(2, 3, 2, s0) SW_BLK(3, 4, 2, s1)
                SW_BLK(4, 5, 3, s0) SW_BLK(5, 6, 3, s1) SW_BLKN(6, 7) SW_LAST(7)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_HE(4), SW_HE(5), SW_HE(6), SW_HE(7), SW_OUTS,
              [sm] "=&v"(sm)
            : SW_INS, SW_AB(0), SW_AB(1), SW_AB(2), SW_AB(3), [s0] "s"(s0), [s1] "s"(s1));
    } else {
        static_assert(R == 4, "rows per lane must be 4, 8 or 16");
        asm(SW_PRO SW_BLK(0, 1, 1, s0) SW_BLK(1, 2, 1, s1) SW_BLKN(2, 3) SW_LAST(3)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_OUTS, [sm] "=&v"(sm)
            : SW_INS, SW_AB(0), SW_AB(1), [s0] "s"(s0), [s1] "s"(s1));
    }
}

// Pre-packed form: w[r] is row r's substitution pair.
template <int R>
__device__ __forceinline__ void rows16_packed(s2* H, s2* E, s2& S, s2& F, s2 diag, const uint32_t* w, u2 go,
                                              u2 ge) {
    s2 hd, t, hgo, es, fs;
    if constexpr (R == 16) {
        asm(SW_PROW SW_BLK0W SW_BLKW(1, 2) SW_BLKW(2, 3) SW_BLKW(3, 4) SW_BLKW(4, 5) SW_BLKW(5, 6) SW_BLKW(6, 7)
                SW_BLKW(7, 8) SW_BLKW(8, 9) SW_BLKW(9, 10) SW_BLKW(10, 11) SW_BLKW(11, 12) SW_BLKW(12, 13)
                    SW_BLKW(13, 14) SW_BLKW(14, 15) SW_LAST(15)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_HE(4), SW_HE(5), SW_HE(6), SW_HE(7), SW_HE(8), SW_HE(9),
              SW_HE(10), SW_HE(11), SW_HE(12), SW_HE(13), SW_HE(14), SW_HE(15), SW_OUTS
            : SW_INS, SW_W(0), SW_W(1), SW_W(2), SW_W(3), SW_W(4), SW_W(5), SW_W(6), SW_W(7), SW_W(8), SW_W(9),
              SW_W(10), SW_W(11), SW_W(12), SW_W(13), SW_W(14), SW_W(15));
    } else if constexpr (R == 8) {
        asm(SW_PROW SW_BLK0W SW_BLKW(1, 2) SW_BLKW(2, 3) SW_BLKW(3, 4) SW_BLKW(4, 5) SW_BLKW(5, 6) SW_BLKW(6, 7)
                SW_LAST(7)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_HE(4), SW_HE(5), SW_HE(6), SW_HE(7), SW_OUTS
            : SW_INS, SW_W(0), SW_W(1), SW_W(2), SW_W(3), SW_W(4), SW_W(5), SW_W(6), SW_W(7));
    } else {
        static_assert(R == 4, "rows per lane must be 4, 8 or 16");
        asm(SW_PROW SW_BLK0W SW_BLKW(1, 2) SW_BLKW(2, 3) SW_LAST(3)
            : SW_HE(0), SW_HE(1), SW_HE(2), SW_HE(3), SW_OUTS
            : SW_INS, SW_W(0), SW_W(1), SW_W(2), SW_W(3));
    }
}

// ------------------------------------------------------------ one pass of one wave
// Rows [p*B*R, (p+1)*B*R) of the query against columns [0, ncols) of the
// wave's pairs.  `lrow` points at this lane's profile rows in LDS, laid out
// [residue][R] (int16).  State lives in registers; only the boundary row
// between passes touches memory.
template <class C, int R, bool COOP>
__device__ __forceinline__ void sweep_pass(const uint8_t* resp, int ncols, int lgB, int b, int s, int p,
                                           int passes, const int16_t* lrow, uint32_t* slot,
                                           typename C::G go, typename C::G ge, typename C::T& S) {
    using T = typename C::T;
    const int B = 1 << lgB;
    const int P = kGroupPairs >> lgB;
    const int nchunks = ncols >> 2;
    const int nsteps = ncols + B - 1;
    const int nloop = (nsteps + 3) >> 2;
    const bool first_lane = (b == 0);
    const bool last_lane = (b == B - 1);
    const bool read_bnd = first_lane && p > 0;
    const bool write_bnd = last_lane && p + 1 < passes;
    const int cstride = P * 4 * C::kWords;        // words per chunk row of the slot
    uint32_t* sbase = slot + s * 4 * C::kWords;

    T H[R], E[R];      // H and E of this lane's rows at the last column done
#pragma unroll
    for (int r = 0; r < R; ++r) { H[r] = C::zero(); E[r] = C::zero(); }
    T diag_top = C::zero();          // H of the row above this lane's block, previous column
    T up_h = C::zero(), up_f = C::zero();   // values shifted in from lane b-1

    // residue stream: this lane works on columns 4c - b .. 4c - b + 3 during loop iteration c
    const int coff = COOP ? ((-b) >> 2) : 0;      // floor((-b)/4)
    const int csh = COOP ? ((-b) & 3) : 0;
    uint2 lo = load_chunk(resp, coff, nchunks);
    uint2 hi = COOP ? load_chunk(resp, coff + 1, nchunks) : make_uint2(0, 0);
    // boundary stream (first lane of a pair, passes after the first)
    T bh[4], bf[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) { bh[u] = C::zero(); bf[u] = C::zero(); }
    if (read_bnd && nchunks > 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) ld_words<C>(sbase + u * C::kWords, bh[u], bf[u]);
    }

    for (int c = 0; c < nloop; ++c) {
        // prefetch next chunk of residues and boundary values
        uint2 nhi = load_chunk(resp, coff + c + (COOP ? 2 : 1), nchunks);
        T nbh[4], nbf[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) { nbh[u] = C::zero(); nbf[u] = C::zero(); }
        if (read_bnd && c + 1 < nchunks) {
            const uint32_t* w = sbase + (int64_t)(c + 1) * cstride;
#pragma unroll
            for (int u = 0; u < 4; ++u) ld_words<C>(w + u * C::kWords, nbh[u], nbf[u]);
        }
        uint32_t ra, rb;
        if (COOP) {
            ra = __builtin_amdgcn_alignbyte(hi.x, lo.x, csh);
            rb = __builtin_amdgcn_alignbyte(hi.y, lo.y, csh);
        } else {
            ra = lo.x;
            rb = lo.y;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = 4 * c + u;
            const int da = (ra >> (8 * u)) & 0xff;
            const int db = (rb >> (8 * u)) & 0xff;
            uint32_t pa[R / 2], pb[R / 2];
            if constexpr (R % 8 == 0) {
                const uint4* qa = reinterpret_cast<const uint4*>(lrow + da * R);
                const uint4* qb = reinterpret_cast<const uint4*>(lrow + db * R);
#pragma unroll
                for (int v = 0; v < R / 8; ++v) {
                    uint4 x = qa[v], y = qb[v];
                    pa[4 * v] = x.x; pa[4 * v + 1] = x.y; pa[4 * v + 2] = x.z; pa[4 * v + 3] = x.w;
                    pb[4 * v] = y.x; pb[4 * v + 1] = y.y; pb[4 * v + 2] = y.z; pb[4 * v + 3] = y.w;
                }
            } else {
                static_assert(R == 4, "rows per lane must be 4 or a multiple of 8");
                const uint2 x = *reinterpret_cast<const uint2*>(lrow + da * R);
                const uint2 y = *reinterpret_cast<const uint2*>(lrow + db * R);
                pa[0] = x.x; pa[1] = x.y;
                pb[0] = y.x; pb[1] = y.y;
            }
            T htop, ftop;
            if (COOP) {
                htop = C::sel(first_lane, bh[u], up_h);
                ftop = C::sel(first_lane, bf[u], up_f);
            } else {
                htop = bh[u];
                ftop = bf[u];
            }
            T F = ftop;
            if constexpr (std::is_same<C, CellI16>::value) {
                rows16_pair<R>(H, E, S, F, diag_top, pa, pb, go, ge);
            } else {
                T diag = diag_top;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    T hd = C::add(diag, C::sm(pa[r >> 1], pb[r >> 1], r));
                    T h = C::mx(C::mx(hd, E[r]), F);
                    S = C::mx(S, hd);
                    diag = H[r];
                    H[r] = h;
                    T hgo = C::gap(h, go);
                    E[r] = C::mx(C::gap(E[r], ge), hgo);
                    F = C::mx(C::gap(F, ge), hgo);
                }
            }
            diag_top = htop;
            const T hbot = H[R - 1];
            if (write_bnd) {
                const int j = t - (B - 1);
                if (j >= 0 && j < ncols)
                    C::put(sbase + (int64_t)(j >> 2) * cstride + (j & 3) * C::kWords, hbot, F);
            }
            if (COOP) {
                up_h = C::shift(hbot);
                up_f = C::shift(F);
            }
        }
        lo = hi;
        hi = nhi;
        if (!COOP) lo = nhi;
#pragma unroll
        for (int u = 0; u < 4; ++u) { bh[u] = nbh[u]; bf[u] = nbf[u]; }
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

template <class C, int R>
__device__ __forceinline__ void run_unit_passes(const SweepArgs& a, int g, int k, int lgB, int q, bool valid,
                                                bool shared_slice, int16_t* lds, int wave, int lane,
                                                uint32_t* slot) {
    using T = typename C::T;
    const int B = 1 << lgB;
    const int P = kGroupPairs >> lgB;
    const int s = lane >> lgB;
    const int b = lane & (B - 1);
    const QDesc Q = a.qd[q];
    const int rows_pp = R << lgB;
    const int passes = (Q.m + rows_pp - 1) / rows_pp;
    GroupRec G{0, 0, 0};
    int ncols = 0;
    if (valid) {
        G = a.groups[g];
        // pairs are sorted by length within the group: the unit's first pair is its widest
        ncols = a.pair_cols[g * kGroupPairs + k * P];
    }
    const int pair = k * P + s;
    const uint8_t* resp = a.image + G.base + pair * 8;
    const int16_t* prof = a.prof + Q.prof_off;
    int16_t* region = shared_slice ? lds : lds + wave * (kNRes * 16 * R);
    const int16_t* lrow = region + b * kNRes * R;
    const typename C::G go = C::gapv(a.go), ge = C::gapv(a.ge);
    T S = C::zero();
    for (int p = 0; p < passes; ++p) {
        if (shared_slice) {
            __syncthreads();
            load_slice<R>(region, prof, Q.mp, p * rows_pp, lgB, threadIdx.x, blockDim.x);
            __syncthreads();
        } else {
            __builtin_amdgcn_wave_barrier();
            load_slice<R>(region, prof, Q.mp, p * rows_pp, lgB, lane, 64);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
        if (valid) {
            if (lgB == 0)
                sweep_pass<C, R, false>(resp, ncols, lgB, b, s, p, passes, lrow, slot, go, ge, S);
            else
                sweep_pass<C, R, true>(resp, ncols, lgB, b, s, p, passes, lrow, slot, go, ge, S);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");   // boundary stores visible to the next pass
    }
    if (!valid) return;
    for (int o = 1; o < B; o <<= 1) S = C::xmax(S, o);
    if (b == 0) {
        const int slot0 = g * kGroupSubjects + 2 * pair;
        const int o0 = a.perm[slot0], o1 = a.perm[slot0 + 1];
        int32_t* out = Q.out ? Q.out : a.scores + Q.out_off;
        if (o0 >= 0) out[o0] = C::lo(S);
        if (o1 >= 0) out[o1] = C::hi(S);
        if (a.rerun != nullptr && (C::lo(S) >= a.sat || C::hi(S) >= a.sat)) {
            const int idx = atomicAdd(a.rerun_count, 1);
            if (idx < a.rerun_cap) a.rerun[idx] = WgItem{g, q, (int16_t)pair, 6, 1, 1};
        }
    }
}

template <class C, int R>
__global__ __launch_bounds__(64 * kWaves) void k_sweep(SweepArgs a) {
    // one shared slice of up to 64*R rows, or four per-wave slices of up to 16*R rows
    __shared__ __attribute__((aligned(16))) int16_t lds[kNRes * 64 * R];
    __shared__ int s_item;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    uint32_t* slot = a.scratch + ((int64_t)(a.slot_base + blockIdx.x) * kWaves + wave) * a.slot_words;
    int n_items = a.n_items;
    if (a.n_items_dev) {
        const int c = min(*a.n_items_dev, a.n_items);
        n_items = c;
    }
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= n_items) break;
        if (a.unit_list) {
            // one unit per workgroup, computed by wave 0 with the whole LDS slice
            const WgItem I = a.items[it];
            run_unit_passes<C, R>(a, I.g0, I.k0, I.lgB, I.q, wave == 0, true, lds, wave, lane, slot);
        } else {
            const WgItem I = a.items[it];
            const int B = 1 << I.lgB;
            int k = I.k0 + wave;
            const int g = I.g0 + (k >> I.lgB) * I.gstep;
            k &= B - 1;
            const bool shared_slice = I.lgB > 4;        // more than 16 lanes per pair
            run_unit_passes<C, R>(a, g, k, I.lgB, I.q, wave < I.count, shared_slice, lds, wave, lane, slot);
        }
    }
}

// ------------------------------------------------------------ query-pair sweep
// Two queries per lane: the two halves of every packed cell are the same
// subject against query a and query b, so a row's substitution pair is one
// dword of a pre-interleaved profile slice and needs no permute.  A wave owns
// P = 64/B subjects of a group (B lanes each, anti-diagonal as above); a group
// has 2B such units.

__device__ __forceinline__ uint32_t load_chunk1(const uint8_t* resp, int c, int nchunks) {
    if (c < 0 || c >= nchunks) return 0x14141414u;
    return *reinterpret_cast<const uint32_t*>(resp + (int64_t)c * kChunkBytes);
}

template <int R, bool COOP>
__device__ __forceinline__ void sweep_pass_q2(const uint8_t* resp, int ncols, int lgB, int b, int s, int p, int passes,
                                              const uint32_t* lrow, uint32_t* slot, u2 go, u2 ge, s2& S) {
    using C = CellI16;
    using T = s2;
    const int B = 1 << lgB;
    const int P = kGroupPairs >> lgB;
    const int nchunks = ncols >> 2;
    const int nsteps = ncols + B - 1;
    const int nloop = (nsteps + 3) >> 2;
    const bool first_lane = (b == 0);
    const bool read_bnd = first_lane && p > 0;
    const bool write_bnd = (b == B - 1) && p + 1 < passes;
    const int cstride = P * 4 * C::kWords;
    uint32_t* sbase = slot + s * 4 * C::kWords;

    T H[R], E[R];      // H and E of this lane's rows at the last column done
#pragma unroll
    for (int r = 0; r < R; ++r) { H[r] = C::zero(); E[r] = C::zero(); }
    T diag_top = C::zero();
    T up_h = C::zero(), up_f = C::zero();
    const int coff = COOP ? ((-b) >> 2) : 0;
    const int csh = COOP ? ((-b) & 3) : 0;
    uint32_t lo = load_chunk1(resp, coff, nchunks);
    uint32_t hi = COOP ? load_chunk1(resp, coff + 1, nchunks) : 0u;
    T bh[4], bf[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) { bh[u] = C::zero(); bf[u] = C::zero(); }
    if (read_bnd && nchunks > 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) ld_words<C>(sbase + u * C::kWords, bh[u], bf[u]);
    }
    for (int c = 0; c < nloop; ++c) {
        const uint32_t nhi = load_chunk1(resp, coff + c + (COOP ? 2 : 1), nchunks);
        T nbh[4], nbf[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) { nbh[u] = C::zero(); nbf[u] = C::zero(); }
        if (read_bnd && c + 1 < nchunks) {
            const uint32_t* w = sbase + (int64_t)(c + 1) * cstride;
#pragma unroll
            for (int u = 0; u < 4; ++u) ld_words<C>(w + u * C::kWords, nbh[u], nbf[u]);
        }
        const uint32_t rr = COOP ? __builtin_amdgcn_alignbyte(hi, lo, csh) : lo;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = 4 * c + u;
            const int d = (rr >> (8 * u)) & 0xff;
            uint32_t w[R];
            if constexpr (R % 4 == 0) {
                const uint4* q = reinterpret_cast<const uint4*>(lrow + d * R);
#pragma unroll
                for (int v = 0; v < R / 4; ++v) {
                    const uint4 x = q[v];
                    w[4 * v] = x.x; w[4 * v + 1] = x.y; w[4 * v + 2] = x.z; w[4 * v + 3] = x.w;
                }
            }
            T htop, ftop;
            if (COOP) {
                htop = C::sel(first_lane, bh[u], up_h);
                ftop = C::sel(first_lane, bf[u], up_f);
            } else {
                htop = bh[u];
                ftop = bf[u];
            }
            T F = ftop;
            rows16_packed<R>(H, E, S, F, diag_top, w, go, ge);
            diag_top = htop;
            const T hbot = H[R - 1];
            if (write_bnd) {
                const int j = t - (B - 1);
                if (j >= 0 && j < ncols)
                    C::put(sbase + (int64_t)(j >> 2) * cstride + (j & 3) * C::kWords, hbot, F);
            }
            if (COOP) {
                up_h = C::shift(hbot);
                up_f = C::shift(F);
            }
        }
        lo = COOP ? hi : nhi;
        hi = nhi;
#pragma unroll
        for (int u = 0; u < 4; ++u) { bh[u] = nbh[u]; bf[u] = nbf[u]; }
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

template <int R>
__device__ __forceinline__ void run_unit_q2(const SweepArgs& a, int g, int k, int lgB, int qp, bool valid,
                                            bool shared_slice, int16_t* lds, int wave, int lane, uint32_t* slot) {
    using T = s2;
    const int B = 1 << lgB;
    const int P = kGroupPairs >> lgB;                   // subjects per unit
    const int s = lane >> lgB;
    const int b = lane & (B - 1);
    const int2 pr = a.qpairs[qp];
    const QDesc Qa = a.qd[pr.x];
    const QDesc Qb = a.qd[pr.y >= 0 ? pr.y : pr.x];
    const int m = max(Qa.m, Qb.m);
    const int rows_pp = R << lgB;
    const int passes = (m + rows_pp - 1) / rows_pp;
    GroupRec G{0, 0, 0};
    int ncols = 0;
    const int su = k * P + s;                           // subject within the group
    if (valid) {
        G = a.groups[g];
        ncols = a.pair_cols[g * kGroupPairs + ((k * P) >> 1)];
    }
    const uint8_t* resp = a.image + G.base + (su >> 1) * 8 + (su & 1) * 4;
    uint32_t* region = reinterpret_cast<uint32_t*>(shared_slice ? lds : lds + wave * (kNRes * 16 * R));
    const uint32_t* lrow = region + b * kNRes * R;
    const u2 go = CellI16::gapv(a.go), ge = CellI16::gapv(a.ge);
    T S = CellI16::zero();
    for (int p = 0; p < passes; ++p) {
        if (shared_slice) {
            __syncthreads();
            load_slice_q2<R>(region, a.prof + Qa.prof_off, Qa.mp, a.prof + Qb.prof_off, Qb.mp, p * rows_pp, lgB,
                             threadIdx.x, blockDim.x);
            __syncthreads();
        } else {
            __builtin_amdgcn_wave_barrier();
            load_slice_q2<R>(region, a.prof + Qa.prof_off, Qa.mp, a.prof + Qb.prof_off, Qb.mp, p * rows_pp, lgB,
                             lane, 64);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
        if (valid) {
            if (lgB == 0)
                sweep_pass_q2<R, false>(resp, ncols, lgB, b, s, p, passes, lrow, slot, go, ge, S);
            else
                sweep_pass_q2<R, true>(resp, ncols, lgB, b, s, p, passes, lrow, slot, go, ge, S);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    }
    if (!valid) return;
    for (int o = 1; o < B; o <<= 1) S = CellI16::xmax(S, o);
    if (b == 0) {
        const int slot0 = g * kGroupSubjects + su;
        const int o = a.perm[slot0];
        if (o >= 0) {
            int32_t* outa = Qa.out ? Qa.out : a.scores + Qa.out_off;
            outa[o] = S.x;
            if (pr.y >= 0) {
                int32_t* outb = Qb.out ? Qb.out : a.scores + Qb.out_off;
                outb[o] = S.y;
            }
        }
        if (a.rerun != nullptr) {
            if (S.x >= a.sat) {
                const int idx = atomicAdd(a.rerun_count, 1);
                if (idx < a.rerun_cap) a.rerun[idx] = WgItem{g, pr.x, (int16_t)(su >> 1), 6, 1, 1};
            }
            if (pr.y >= 0 && S.y >= a.sat) {
                const int idx = atomicAdd(a.rerun_count, 1);
                if (idx < a.rerun_cap) a.rerun[idx] = WgItem{g, pr.y, (int16_t)(su >> 1), 6, 1, 1};
            }
        }
    }
}

template <int R>
__global__ __launch_bounds__(64 * kWaves) void k_sweep_q2(SweepArgs a) {
    __shared__ __attribute__((aligned(16))) int16_t lds[kNRes * 64 * R];
    __shared__ int s_item;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    uint32_t* slot = a.scratch + ((int64_t)(a.slot_base + blockIdx.x) * kWaves + wave) * a.slot_words;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= a.n_items) break;
        const WgItem I = a.items[it];
        const int units = 2 << I.lgB;                   // units per group
        int k = I.k0 + wave;
        const int g = I.g0 + (k / units) * I.gstep;
        k %= units;
        const bool shared_slice = I.lgB > 3;            // more than 8 lanes per subject
        run_unit_q2<R>(a, g, k, I.lgB, I.q, wave < I.count, shared_slice, lds, wave, lane, slot);
    }
}

// ------------------------------------------------------------ query profile
// prof[d][i] = SM(Q[i], d) for d < 20 and i < m; kPadScore elsewhere.  One
// staging buffer holds the 20x20 matrix followed by the query codes.
// Thread 0 also zeroes the launch counters (they are consumed by later kernels
// on the same stream).
__global__ void k_profile(const int8_t* stage, const QDesc* qd, int nq, const int64_t* qoff,
                          int16_t* prof, int32_t* counters, int ncounters) {
    const int q = blockIdx.y;
    if (q == 0 && blockIdx.x == 0 && threadIdx.x < ncounters) counters[threadIdx.x] = 0;
    if (q >= nq) return;
    const QDesc Q = qd[q];
    const int8_t* sm = stage;
    const int8_t* query = stage + 400 + qoff[q];
    const int64_t total = (int64_t)kNRes * Q.mp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int d = (int)(e / Q.mp);
        const int i = (int)(e - (int64_t)d * Q.mp);
        int16_t v = kPadScore;
        if (d < 20 && i < Q.m) v = sm[query[i] * 20 + d];
        prof[Q.prof_off + e] = v;
    }
}

// ------------------------------------------------------------ database interleave
// One thread per output dword: 4 consecutive columns of one subject.
__global__ void k_interleave(const int8_t* res, const int64_t* soff, const int32_t* slen, int64_t n,
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
        uint32_t word = 0x14141414u;
        if (sidx < n) {
            const int64_t off = soff[sidx];
            const int len = slen[sidx];
            word = 0;
            for (int kk = 0; kk < 4; ++kk) {
                const int64_t col = 4 * c + kk;
                uint32_t v = kPadCode;
                if (col < len) {
                    const int r = res[off + col];
                    if (r < 0 || r >= 20) { atomicOr(err, 1); v = kPadCode; }
                    else v = (uint32_t)r;
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

__global__ __launch_bounds__(kTopkThreads) void k_topk(const int32_t* scores, int64_t n, int64_t row_stride, int k,
                                                       int32_t* top_s, int64_t* top_i) {
    __shared__ int hist[256];
    __shared__ int s_digit, s_rank;
    __shared__ int c_gt, c_eq;
    __shared__ int wave_cnt[kTopkThreads / 64];
    __shared__ int cand_s[1024];
    __shared__ int64_t cand_i[1024];
    const int tid = threadIdx.x;
    const int32_t* row = scores + (int64_t)blockIdx.x * row_stride;
    int32_t* outs = top_s + (int64_t)blockIdx.x * k;
    int64_t* outi = top_i + (int64_t)blockIdx.x * k;
    const int take = (int)min<int64_t>((int64_t)k, n);

    uint32_t prefix = 0, mask = 0;
    int rank = take;                 // rank of the threshold among scores matching the prefix
    if (take > 0 && take < n) {
        for (int shift = 24; shift >= 0; shift -= 8) {
            for (int i = tid; i < 256; i += kTopkThreads) hist[i] = 0;
            __syncthreads();
            for (int64_t i = tid; i < n; i += kTopkThreads) {
                const uint32_t v = (uint32_t)row[i];
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
    const int T = (take > 0 && take < n) ? (int)prefix : -1;   // take == n: every score qualifies
    const int need_eq = (take > 0 && take < n) ? rank : 0;
    if (tid == 0) { c_gt = 0; c_eq = 0; }
    __syncthreads();
    for (int64_t base = 0; base < n && take > 0; base += kTopkThreads) {
        const int64_t i = base + tid;
        const int v = i < n ? row[i] : -2;
        const bool gt = v > T;
        const bool eq = (v == T) && (T >= 0);
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
        if (i >= take) { cand_s[i] = -1; cand_i[i] = INT64_MAX; }
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
        if (i < take) { outs[i] = cand_s[i]; outi[i] = cand_i[i]; }
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

hipError_t sweep_occupancy(bool i16, int R, int* blocks_per_cu) {
    const void* k = sweep_kernel(i16, R);
    if (!k) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, 64 * kWaves, 0);
}

hipError_t launch_profile(const int8_t* stage, const QDesc* qd, int nq, const int64_t* qoff, int16_t* prof,
                          int32_t* counters, int ncounters, int max_mp, hipStream_t st) {
    const int bx = (int)std::min<int64_t>(((int64_t)kNRes * max_mp + 255) / 256, 1024);
    hipLaunchKernelGGL(k_profile, dim3(bx, std::max(nq, 1)), dim3(256), 0, st, stage, qd, nq, qoff, prof,
                       counters, ncounters);
    return hipGetLastError();
}

hipError_t launch_interleave(const int8_t* res, const int64_t* soff, const int32_t* slen, int64_t n,
                             const GroupRec* groups, const int64_t* gdw, int ngroups, uint32_t* image,
                             int64_t total_dw, int32_t* err, hipStream_t st) {
    const int64_t blocks = std::min<int64_t>((total_dw + 255) / 256, 65536);
    hipLaunchKernelGGL(k_interleave, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, res, soff, slen, n,
                       groups, gdw, ngroups, image, total_dw, err);
    return hipGetLastError();
}

hipError_t launch_topk(const int32_t* scores, int64_t n, int64_t row_stride, int rows, int k, int32_t* top_s,
                       int64_t* top_i, hipStream_t st) {
    hipLaunchKernelGGL(k_topk, dim3(rows), dim3(kTopkThreads), 0, st, scores, n, row_stride, k, top_s, top_i);
    return hipGetLastError();
}

hipError_t launch_fill(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace sw
