// Device code of the batched Smith-Waterman library, written for gfx950.
//
// What is computed per pair (query q of length m, reference r of length n):
// the local-alignment recurrence with affine gaps over the whole m x n matrix
// (the paper, section "Load balancing techniques": the aligner fills the
// entire matrix, so a pair costs m*n), the best score S, the first cell of S
// in (query, reference) lexicographic order, and the start found by running
// the same recurrence over the reversed prefixes (first reversed cell that
// reaches S).  All arithmetic is exact int32.
//
// Cell update of the int32 paths (about 10 VALU instructions per cell):
//   d  = H[i-1][j-1] + s(q_i, r_j)           profile nibble (v_bfe) + add3 with -bias
//   H  = max3(d, E[i][j], F[i][j])           E, F >= 0, so H >= 0 is the local floor
//   hg = sat(H - go)                         v_sub_u32 clamp
//   E[i][j+1] = max(E[i][j] - ge, hg)        hg >= 0 keeps E >= 0
//   F[i+1][j] = max(F[i][j] - ge, hg)
//   K[r] = max(K[r], H << TB | tag(j))       per-row best with the earliest column
// Keeping E and F saturated at 0 leaves H exactly as in the textbook
// recurrence: by induction E_sat = max(E, 0), and H only uses max(0, E).
//
// Work decomposition.  Pairs up to 1024 residues get one lane each, longer
// ones up to 2048 a group of 8 lanes, longer still a whole wave (the limits
// are tunable; a middle tier of 16-lane groups is off by default).  A lane
// keeps R query rows in registers and sweeps the reference in chunks of 8
// columns; a group of P lanes covers a super-strip of P R rows as a
// wavefront, and super-strips hand their bottom row to the next one through a
// per-block scratch slot.  Scores come from a per-lane query profile in LDS.
// The one-, 8- and 16-lane paths first run a packed 16-bit pass (two cells per
// instruction) that only finds the best score and the super-strip holding its
// first cell, then recompute that super-strip in int32 with cell trackers;
// the whole-wave path ("wide": any length, two dwords per boundary cell,
// 12-bit column tags folded every 4096 columns) runs in int32 throughout.

#include <algorithm>
#include <type_traits>

#include "sw_internal.h"

namespace swk {

// ------------------------------------------------------------------ alphabet
// The library's own copy of BLOSUM62 (NCBI symbol order) and its symbol order
// for packing: the 16 most frequent amino acids get codes 0..15 so that their
// high bit is 0.
static constexpr char kNcbiOrder[kNumSym + 1] = "ARNDCQEGHILKMFPSTWYVBZX*";
static constexpr char kCodeOrder[kNumSym + 1] = "LAGVIKSEDRTFNPQYHMCWBZX*";
static constexpr int8_t kBlosum62Ncbi[kNumSym][kNumSym] = {
    // A   R   N   D   C   Q   E   G   H   I   L   K   M   F   P   S   T   W   Y   V   B   Z   X   *
    { 4, -1, -2, -2,  0, -1, -1,  0, -2, -1, -1, -1, -1, -2, -1,  1,  0, -3, -2,  0, -2, -1,  0, -4},  // A
    {-1,  5,  0, -2, -3,  1,  0, -2,  0, -3, -2,  2, -1, -3, -2, -1, -1, -3, -2, -3, -1,  0, -1, -4},  // R
    {-2,  0,  6,  1, -3,  0,  0,  0,  1, -3, -3,  0, -2, -3, -2,  1,  0, -4, -2, -3,  3,  0, -1, -4},  // N
    {-2, -2,  1,  6, -3,  0,  2, -1, -1, -3, -4, -1, -3, -3, -1,  0, -1, -4, -3, -3,  4,  1, -1, -4},  // D
    { 0, -3, -3, -3,  9, -3, -4, -3, -3, -1, -1, -3, -1, -2, -3, -1, -1, -2, -2, -1, -3, -3, -2, -4},  // C
    {-1,  1,  0,  0, -3,  5,  2, -2,  0, -3, -2,  1,  0, -3, -1,  0, -1, -2, -1, -2,  0,  3, -1, -4},  // Q
    {-1,  0,  0,  2, -4,  2,  5, -2,  0, -3, -3,  1, -2, -3, -1,  0, -1, -3, -2, -2,  1,  4, -1, -4},  // E
    { 0, -2,  0, -1, -3, -2, -2,  6, -2, -4, -4, -2, -3, -3, -2,  0, -2, -2, -3, -3, -1, -2, -1, -4},  // G
    {-2,  0,  1, -1, -3,  0,  0, -2,  8, -3, -3, -1, -2, -1, -2, -1, -2, -2,  2, -3,  0,  0, -1, -4},  // H
    {-1, -3, -3, -3, -1, -3, -3, -4, -3,  4,  2, -3,  1,  0, -3, -2, -1, -3, -1,  3, -3, -3, -1, -4},  // I
    {-1, -2, -3, -4, -1, -2, -3, -4, -3,  2,  4, -2,  2,  0, -3, -2, -1, -2, -1,  1, -4, -3, -1, -4},  // L
    {-1,  2,  0, -1, -3,  1,  1, -2, -1, -3, -2,  5, -1, -3, -1,  0, -1, -3, -2, -2,  0,  1, -1, -4},  // K
    {-1, -1, -2, -3, -1,  0, -2, -3, -2,  1,  2, -1,  5,  0, -2, -1, -1, -1, -1,  1, -3, -1, -1, -4},  // M
    {-2, -3, -3, -3, -2, -3, -3, -3, -1,  0,  0, -3,  0,  6, -4, -2, -2,  1,  3, -1, -3, -3, -1, -4},  // F
    {-1, -2, -2, -1, -3, -1, -1, -2, -2, -3, -3, -1, -2, -4,  7, -1, -1, -4, -3, -2, -2, -1, -2, -4},  // P
    { 1, -1,  1,  0, -1,  0,  0,  0, -1, -2, -2,  0, -1, -2, -1,  4,  1, -3, -2, -2,  0,  0,  0, -4},  // S
    { 0, -1,  0, -1, -1, -1, -1, -2, -2, -1, -1, -1, -1, -2, -1,  1,  5, -2, -2,  0, -1, -1,  0, -4},  // T
    {-3, -3, -4, -4, -2, -2, -3, -2, -2, -3, -2, -3, -1,  1, -4, -3, -2, 11,  2, -3, -4, -3, -2, -4},  // W
    {-2, -2, -2, -3, -2, -1, -2, -3,  2, -1, -1, -2, -1,  3, -3, -2, -2,  2,  7, -1, -3, -2, -1, -4},  // Y
    { 0, -3, -3, -3, -1, -2, -2, -3, -3,  3,  1, -2,  1, -1, -2, -2,  0, -3, -1,  4, -3, -2, -1, -4},  // V
    {-2, -1,  3,  4, -3,  0,  1, -1,  0, -3, -4,  0, -3, -3, -2,  0, -1, -4, -3, -3,  4,  1, -1, -4},  // B
    {-1,  0,  0,  1, -3,  3,  4, -2,  0, -3, -3,  1, -1, -3, -1,  0, -1, -3, -2, -2,  1,  4, -1, -4},  // Z
    { 0, -1, -1, -1, -2, -1, -1, -1, -1, -1, -1, -1, -1, -1, -2,  0,  0, -2, -1, -1, -1, -1, -1, -4},  // X
    {-4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4,  1},  // *
};

static constexpr int ncbi_index(char c)
{
    for (int k = 0; k < kNumSym; ++k)
        if (kNcbiOrder[k] == c) return k;
    return -1;
}

// Offset that makes every BLOSUM62 score non-negative (the minimum is -4).
constexpr int kScoreBias = 4;

struct CodeTables {
    uint32_t tabb[kNumCodes][8];  // row c: bytes s(c, x) + kScoreBias for x = 0..31 (pad and unused: 0)
    uint8_t ascii[256];           // ASCII -> code, 0xFF if not a symbol
};

static constexpr CodeTables make_tables()
{
    CodeTables t{};
    for (int a = 0; a < kNumCodes; ++a)
        for (int w = 0; w < 8; ++w) {
            uint32_t wordb = 0;
            for (int k = 0; k < 4; ++k) {
                int b = 4 * w + k;
                int vb = 0;
                if (a < kNumSym && b < kNumSym)
                    vb = kBlosum62Ncbi[ncbi_index(kCodeOrder[a])][ncbi_index(kCodeOrder[b])] + kScoreBias;
                wordb |= (uint32_t)(uint8_t)vb << (8 * k);
            }
            t.tabb[a][w] = wordb;
        }
    for (int c = 0; c < 256; ++c) t.ascii[c] = 0xFF;
    for (int a = 0; a < kNumSym; ++a) t.ascii[(unsigned char)kCodeOrder[a]] = (uint8_t)a;
    return t;
}

static constexpr CodeTables kTables = make_tables();
__constant__ CodeTables c_tables = kTables;

void matrix_ncbi(int8_t out[kNumSym * kNumSym], char letters[kNumSym + 1])
{
    for (int a = 0; a < kNumSym; ++a)
        for (int b = 0; b < kNumSym; ++b) out[a * kNumSym + b] = kBlosum62Ncbi[a][b];
    for (int a = 0; a <= kNumSym; ++a) letters[a] = kNcbiOrder[a];
}

const char* code_order() { return kCodeOrder; }

// ------------------------------------------------------------------ packed residues
// A sequence view: residues B + x for x >= -256 addressed with 32-bit offsets
// from the 256-residue block before the one holding B, in both planes.
struct SeqView {
    const uint32_t* nib;
    const uint32_t* hib;
    int off;
};

__device__ __forceinline__ const uint32_t* high_plane(const uint32_t* nib_plane, const PackedHeader* h)
{
    return nib_plane + h->n_blocks * 32;
}

__device__ __forceinline__ SeqView seq_view(const uint32_t* __restrict__ nib_plane, const PackedHeader* h, int64_t B)
{
    const int64_t q = B + kGuardRes;
    SeqView v;
    v.nib = nib_plane + ((q >> 8) - 1) * 32;
    v.hib = high_plane(nib_plane, h) + ((q >> 8) - 1) * 8;
    v.off = (int)(q & 255) + 256;
    return v;
}

// Codes of the 8 residues B+x .. B+x+7: nibble k of nw, bit k of hw.
__device__ __forceinline__ void window8(const SeqView& v, int x, uint32_t& nw, uint32_t& hw)
{
    const int q = v.off + x;
    const uint32_t a0 = v.nib[q >> 3], a1 = v.nib[(q >> 3) + 1];
    nw = __builtin_amdgcn_alignbit(a1, a0, (uint32_t)(q & 7) * 4u);
    const uint32_t b0 = v.hib[q >> 5], b1 = v.hib[(q >> 5) + 1];
    hw = __builtin_amdgcn_alignbit(b1, b0, (uint32_t)(q & 31));
}

// Code of the single residue B + x.
__device__ __forceinline__ uint32_t code_at(const SeqView& v, int x)
{
    const int q = v.off + x;
    return ((v.nib[q >> 3] >> ((q & 7) * 4)) & 15u) | (((v.hib[q >> 5] >> (q & 31)) & 1u) << 4);
}

// Codes of R consecutive rows starting at `row0`, read forwards from the view
// base (REV: backwards).  Rows >= M get the pad code.
template <int R, bool REV>
__device__ __forceinline__ void row_codes(const SeqView& qv, int row0, int M, uint32_t (&qc)[R])
{
    const bool any = row0 < M;
    const int x = !any ? 0 : (REV ? -row0 - (R - 1) : row0);
#pragma unroll
    for (int k8 = 0; k8 < R / 8; ++k8) {
        uint32_t nw, hw;
        window8(qv, x + 8 * k8, nw, hw);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int idx = 8 * k8 + k;                 // window position
            const int r = REV ? (R - 1 - idx) : idx;    // row within the strip
            const uint32_t c = ((nw >> (4 * k)) & 15u) | (((hw >> k) & 1u) << 4);
            qc[r] = (row0 + r < M) ? c : (uint32_t)kPadCode;
        }
    }
}

// ------------------------------------------------------------------ query profile in LDS
// Layout [code][lane][R/2 bytes]: lane l's scores for its R rows against a
// reference residue `code`, plus kScoreBias so that each fits 4 bits (BLOSUM62
// spans -4..11), padding 0.  Dword j of an entry holds rows 4j .. 4j+3 in its
// low half and rows 4(j + R/8) .. in its high half, one nibble per row in row
// order: for R = 16, dword 0 = rows 0-3 | 8-11 and dword 1 = rows 4-7 | 12-15,
// so the packed pass finds the rows of both halves of a register pair in the
// same bit positions.  A wave's reads of one row of the layout are contiguous
// in lane order, so the 4- or 8-byte reads are conflict-free whatever codes
// the lanes hold.  At 8 bytes per lane and code (R = 16) the profile takes
// 12.8 KB per wave, which leaves room for two waves per SIMD.
constexpr int prof_bytes(int R) { return R / 2; }

// 4 bytes, each below 16, as 4 nibbles in the low 16 bits.
__device__ __forceinline__ uint32_t nib4(uint32_t b) { return b | (b >> 4); }  // bytes 0 and 2 hold them

template <int R>
__device__ __forceinline__ void build_profile(uint8_t* prof, int lane, const uint32_t (&qc)[R])
{
    uint32_t sel[R / 4][3];
#pragma unroll
    for (int w = 0; w < R / 4; ++w) {
        uint32_t s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t c = qc[4 * w + i];
            const uint32_t g = c >> 3, idx = c & 7u;
            s0 |= (g == 0 ? idx : 12u) << (8 * i);   // selector 12 -> byte 0x00
            s1 |= (g == 1 ? idx : 12u) << (8 * i);
            s2 |= (g == 2 ? idx : 12u) << (8 * i);
        }
        sel[w][0] = s0;
        sel[w][1] = s1;
        sel[w][2] = s2;
    }
    uint8_t* base = prof + lane * prof_bytes(R);
    // four codes per trip, so that their table loads go out together
#pragma unroll 4
    for (int c = 0; c < kNumSym; ++c) {
        const uint32_t* t = c_tables.tabb[c];
        const uint32_t t0 = t[0], t1 = t[1], t2 = t[2], t3 = t[3], t4 = t[4], t5 = t[5];
        uint32_t v[R / 4];  // rows 4w .. 4w+3, one byte each
#pragma unroll
        for (int w = 0; w < R / 4; ++w)
            v[w] = nib4(__builtin_amdgcn_perm(t1, t0, sel[w][0]) | __builtin_amdgcn_perm(t3, t2, sel[w][1]) |
                        __builtin_amdgcn_perm(t5, t4, sel[w][2]));
        uint8_t* dst = base + c * (kWave * prof_bytes(R));
        // dword j: nibbles of row group j (low half) and j + R/8 (high half)
        if constexpr (R == 8) {
            *reinterpret_cast<uint32_t*>(dst) = __builtin_amdgcn_perm(v[1], v[0], 0x06040200u);
        } else {
            *reinterpret_cast<uint2*>(dst) = make_uint2(__builtin_amdgcn_perm(v[2], v[0], 0x06040200u),
                                                        __builtin_amdgcn_perm(v[3], v[1], 0x06040200u));
        }
    }
    uint8_t* dst = base + kPadCode * (kWave * prof_bytes(R));
    if constexpr (R == 8)
        *reinterpret_cast<uint32_t*>(dst) = 0u;
    else
        *reinterpret_cast<uint2*>(dst) = make_uint2(0u, 0u);
}

template <int R>
__device__ __forceinline__ void load_profile(const uint8_t* prof_lane, uint32_t code, uint32_t (&w)[R / 8])
{
    const uint8_t* p = prof_lane + code * (uint32_t)(kWave * prof_bytes(R));
    if constexpr (R == 8) {
        w[0] = *reinterpret_cast<const uint32_t*>(p);
    } else {
        const uint2 v = *reinterpret_cast<const uint2*>(p);
        w[0] = v.x;
        w[1] = v.y;
    }
}

// Biased score (0..15) of row r in a profile entry.
template <int R, int r>
__device__ __forceinline__ uint32_t nib_score(const uint32_t (&w)[R / 8])
{
    constexpr int grp = r >> 2, j = grp % (R / 8), half = grp / (R / 8);
    return __builtin_amdgcn_ubfe(w[j], 16 * half + 4 * (r & 3), 4);
}

// ------------------------------------------------------------------ the cell update
// Hides what the compiler knows about the value's range (no instruction).
// E and F are never negative; once the compiler proves that, it splits
// max(max(d, E), F) into a signed and an unsigned max instead of one
// v_max3_i32.
__device__ __forceinline__ void opaque(int& v) { asm("" : "+v"(v)); }
__device__ __forceinline__ void opaque(uint32_t& v) { asm("" : "+v"(v)); }

template <int R, int I>
struct RowUnroll {
    template <int TB>
    static __device__ __forceinline__ void run(int (&H)[R], int (&E)[R], uint32_t (&K)[R],
                                               const uint32_t (&w)[R / 8], int& d, int& F,
                                               uint32_t tag, uint32_t go, int ge)
    {
        int dn = 0;
        if constexpr (I + 1 < R) dn = H[I] + (int)nib_score<R, I + 1>(w) - kScoreBias;
        const int h = max(max(d, E[I]), F);
        H[I] = h;
        const int hg = (int)__builtin_elementwise_sub_sat((uint32_t)h, go);
        E[I] = max(E[I] - ge, hg);
        F = max(F - ge, hg);
        opaque(E[I]);
        opaque(F);
        K[I] = max(K[I], ((uint32_t)h << TB) | tag);
        d = dn;
        if constexpr (I + 1 < R) RowUnroll<R, I + 1>::template run<TB>(H, E, K, w, d, F, tag, go, ge);
    }
};

// The same update keeping only a running maximum of H over the lane's rows
// (the scan of the whole-wave path: one max per cell instead of a tracker).
template <int R, int I>
struct RowScan {
    static __device__ __forceinline__ void run(int (&H)[R], int (&E)[R], int& mx, const uint32_t (&w)[R / 8], int& d,
                                               int& F, uint32_t go, int ge)
    {
        int dn = 0;
        if constexpr (I + 1 < R) dn = H[I] + (int)nib_score<R, I + 1>(w) - kScoreBias;
        const int h = max(max(d, E[I]), F);
        H[I] = h;
        const int hg = (int)__builtin_elementwise_sub_sat((uint32_t)h, go);
        E[I] = max(E[I] - ge, hg);
        F = max(F - ge, hg);
        opaque(E[I]);
        opaque(F);
        mx = max(mx, h);
        d = dn;
        if constexpr (I + 1 < R) RowScan<R, I + 1>::run(H, E, mx, w, d, F, go, ge);
    }
};

// One column of a lane's R rows.  hdiag = H[row0-1][j-1]; F enters as
// F[row0][j] and leaves as F[row0+R][j].
template <int R, int TB>
__device__ __forceinline__ void column_step(int (&H)[R], int (&E)[R], uint32_t (&K)[R],
                                            const uint32_t (&w)[R / 8], int hdiag, int& F,
                                            uint32_t tag, uint32_t go, int ge)
{
    int d = hdiag + (int)nib_score<R, 0>(w) - kScoreBias;
    RowUnroll<R, 0>::template run<TB>(H, E, K, w, d, F, tag, go, ge);
}

template <int R>
__device__ __forceinline__ void column_scan(int (&H)[R], int (&E)[R], int& mx, const uint32_t (&w)[R / 8], int hdiag,
                                            int& F, uint32_t go, int ge)
{
    int d = hdiag + (int)nib_score<R, 0>(w) - kScoreBias;
    RowScan<R, 0>::run(H, E, mx, w, d, F, go, ge);
}

// ------------------------------------------------------------------ wave helpers
__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <int CTRL>
__device__ __forceinline__ int dpp_mov(int old, int src)
{
    return __builtin_amdgcn_update_dpp(old, src, CTRL, 0xF, 0xF, false);
}
constexpr int kWaveShr1 = 0x138;  // lane l <- lane l-1; lane 0 keeps `old`
constexpr int kWaveShl1 = 0x130;  // lane l <- lane l+1; lane 63 keeps `old`

__device__ __forceinline__ void block_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

struct Best {
    int s, i, j;
};

// ------------------------------------------------------------------ group sweep
// A group of P lanes (P = 1, 16 or 64) aligns one pair: rows [0, M) x columns
// [0, N).  Row i reads query position Q0 + i (REV: Q0 - i), column j reads
// reference position R0 + j (REV: R0 - j).  Super-strip ss covers rows
// [ss P R, (ss+1) P R); lane u of the group owns rows ss P R + u R + [0, R)
// and at step t processes the 8-column chunk c = t - u.  The bottom row of
// that chunk reaches lane u+1 through the LDS exchange buffer (written at the
// end of step t, read at the start of step t+1 by the same wave, so no
// barrier is needed); lane P-1 hands it to the next super-strip through the
// block's scratch slot, laid out [chunk][group][8 columns].  Boundary cells
// are (H | F << 16) in the narrow variant and (H, F) in the wide one.
// Forward: the best score and its first cell.  REV: the group stops after the
// first super-strip whose rows reach `target`.
template <int P>
__device__ __forceinline__ Best group_best(Best b)
{
#pragma unroll
    for (int o = 1; o < P; o <<= 1) {
        const int s = __shfl_xor(b.s, o, kWave), i = __shfl_xor(b.i, o, kWave), j = __shfl_xor(b.j, o, kWave);
        if (s > b.s || (s == b.s && s > 0 && (i < b.i || (i == b.i && j < b.j)))) {
            b.s = s;
            b.i = i;
            b.j = j;
        }
    }
    return b;
}

// Words of one boundary-row buffer of a block slot for groups of P lanes
// (narrow cells, layout [chunk][group][8 cells]); the packed pass rotates
// three of them.
__host__ __device__ constexpr int64_t boundary_buf_words(int P)
{
    return (P == 1 ? (int64_t)kMaxInterChunks : (int64_t)(kMaxP16Len / 8)) * (kWave / P) * 8;
}

// Boundary buffer of a slot that holds a one-lane forward pass's kept rows
// (after a ring of four); the slot takes kKeptBuf + 1 buffers of such groups.
constexpr int kKeptBuf = 4;

// The same for N columns: a whole wave also runs the start passes of longer
// pairs in narrow cells (one group, one word per column, rounded to 256
// bytes); three such buffers of 65,536 columns fill the least slot.
__host__ __device__ constexpr int64_t narrow_buf_words(int P, int N)
{
    return P == 64 && N > kMaxP16Len ? ((((int64_t)N + 7) / 8) * 8 + 63) & ~(int64_t)63 : boundary_buf_words(P);
}

// ONE: sweep only super-strip `one_ss` of each group (it may differ between
// groups; -1 for none), reading its input row from boundary buffer `one_buf`
// of the slot and writing nothing: the exact-cell pass after the packed
// score pass.
// The top boundary of a pair's first super-strip: read with a zero stride by
// every lane (never written; one chunk of the widest boundary format).
__device__ uint4 g_zero_row[4];

// Words of one boundary-row buffer of the whole-wave path for n columns: one
// group, H and F of every column, rounded to 256 bytes; its scan rotates
// three of them, a pair too long for three in a slot runs the in-place sweep.
__host__ __device__ constexpr int64_t wide_buf_words(int n) { return (((int64_t)(n + 7) / 8) * 16 + 63) & ~(int64_t)63; }
constexpr int64_t kWideBufWords = wide_buf_words(SW_MAX_SEQ_LEN);

// Result of a score-only pass: the super-strip whose int32 recompute gives the
// exact cells, and the boundary buffer that holds its input row.
struct StripPick {
    int s;    // forward: best score (0 if none)
    int ss;   // super-strip to recompute, -1 if none
    int buf;  // boundary buffer holding its input row
};

// SCAN (whole-wave path): keep only the running maximum of each super-strip,
// read and write separate boundary buffers (three of wide_buf_words(N) each,
// rotated as in the packed pass) and report through *pick the super-strip to
// recompute with ONE (same N, so the same buffers):
// forward, the first one that reaches the best score, its input row kept; REV,
// the first one whose maximum reaches `target`.  Padding cells stay below the
// pair's maximum, so they cannot change either choice.
//
// A scan may start at super-strip `ss0` > 0, its input row in buffer `buf0`
// (the forward scan that continues a packed pass which ran out of 16 bits).
template <int R, int P, bool REV, bool WIDE, bool ONE = false, bool SCAN = false>
__device__ __forceinline__ Best group_sweep(const Args& a, uint8_t* prof, uint4* xbuf, uint32_t* __restrict__ slot,
                            int64_t Q0, int M, int64_t R0, int N, int target, int one_ss = -1, int one_buf = 0,
                            StripPick* pick_out = nullptr, int ss0 = 0, int buf0 = 0)
{
    static_assert(!SCAN || (WIDE && !ONE), "the scan is the whole-wave path's score pass");
    const int64_t BUFW = WIDE ? wide_buf_words(N) : narrow_buf_words(P, N);
    constexpr int TB = WIDE ? 12 : 16;  // tag bits of the per-row trackers
    constexpr int SW = WIDE ? 4 : 2;    // uint4 per boundary chunk of 8 columns
    constexpr int G = kWave / P;        // groups per wave
    const int lane = threadIdx.x & (kWave - 1);
    const int u = lane % P, g = lane / P;
    const uint8_t* prof_lane = prof + lane * prof_bytes(R);
    const uint32_t go = (uint32_t)a.go;
    const int ge = a.ge;
    Best b{0, -1, -1};  // this lane's rows only
    const int all_ss = (M > 0 && N > 0) ? (M + P * R - 1) / (P * R) : 0;
    const int my_ss = ONE ? (one_ss >= 0 && one_ss < all_ss ? 1 : 0) : all_ss;
    const int my_chunks = (N + 7) / 8;
    const int wss = uni(wave_max(my_ss));
    const int wc = uni(wave_max(my_ss > 0 ? my_chunks : 0));
    bool done = my_ss == 0 || (REV && target <= 0 && !ONE);
    const SeqView qv = seq_view(a.qblk, a.qhdr, Q0);
    const SeqView rv = seq_view(a.rblk, a.rhdr, R0);
    uint4* slot4 = reinterpret_cast<uint4*>(slot + (ONE ? (int64_t)min(max(one_buf, 0), 2) * BUFW : 0)) + SW * g;
    // SCAN: boundary buffers input, output, kept (uniform in the group)
    int bi = 0, bo = 1, bk = 2;
    if constexpr (SCAN) {
        bi = buf0;
        bo = buf0 == 0 ? 1 : 0;
        bk = 3 - bi - bo;
    }
    StripPick pick{0, -1, 0};
    uint4* x_mine = xbuf + SW * lane;
    const uint4* x_up = xbuf + SW * (lane > 0 ? lane - 1 : 0);

#pragma unroll 1
    for (int ss = SCAN ? ss0 : 0; ss < wss; ++ss) {
        if (__ballot(!done && ss < my_ss) == 0) break;
        const bool gact = !done && ss < my_ss;
        const int sv = ONE ? one_ss : ss;  // super-strip index
        const int row0 = sv * P * R + u * R;
        {
            uint32_t qc[R];
            row_codes<R, REV>(qv, gact ? row0 : M, M, qc);
            build_profile<R>(prof, lane, qc);
        }
        int H[R], E[R];
        uint32_t K[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            H[r] = 0;
            E[r] = 0;
            K[r] = 0;
        }
        int hdiag = 0;
        int mx = 0;  // SCAN: maximum of this lane's cells in the super-strip
        const bool read_top = sv > 0;                    // uniform within the group
        const bool write_next = !ONE && ss + 1 < my_ss;  // uniform within the group

        // wide: fold the 4096-column trackers into this lane's (score, row,
        // column), score descending, then row, then column ascending.  Tags
        // count steps: column = 8 t + k - 8 u.
        auto fold = [&](int tcol_base) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int sc = (int)(K[r] >> 12);
                const int row = row0 + r;
                if (gact && row < M && sc > 0 && (sc > b.s || (sc == b.s && row < b.i))) {
                    b.s = sc;
                    b.i = row;
                    b.j = tcol_base + 4095 - (int)(K[r] & 4095u) - 8 * u;
                }
                K[r] = 0;
            }
        };
        auto chunk_x = [&](int c) -> int {
            return (c < 0 || 8 * c >= N) ? 0 : (REV ? -8 * c - 7 : 8 * c);
        };
        const int T = wc + P - 1;
        // Software pipeline: the global loads of chunk c+1 (reference window,
        // and for lane 0 the boundary row from the slot) are issued at the
        // start of chunk c, and the profile words of column k+1 are read from
        // LDS before column k is computed, so neither latency sits in front of
        // the cell updates.  Idle steps (before the first or past the last
        // chunk) still load, so their indexes are kept inside the pair.
        // No value of a load is used in the iteration that issues it (a
        // select on it, or the window's alignment, would wait for the load
        // right there): the first super-strip reads a zero row with stride 0,
        // padding columns read the last real chunk (real cells of the row
        // above, so padding stays below the pair's maximum), lanes u > 0
        // take the row from lane u - 1 instead, and the window words are
        // aligned where they are used.
        const uint4* rd4 = SCAN ? reinterpret_cast<const uint4*>(slot + bi * BUFW) + SW * g : slot4;
        uint4* wr4 = SCAN ? reinterpret_cast<uint4*>(slot + bo * BUFW) + SW * g : slot4;
        const uint4* in4 = read_top ? rd4 : g_zero_row;
        const int in_stride = read_top ? G * SW : 0;
        uint4 tc_n[SW];
        uint32_t na_n, nb_n, ha_n, hb_n;
        int q_n;
        auto fetch = [&](int cn) {
            const int cc = min(max(cn, 0), max(my_chunks - 1, 0));
#pragma unroll
            for (int w = 0; w < SW; ++w) tc_n[w] = in4[cc * in_stride + w];
            const int q = rv.off + chunk_x(cn);
            na_n = rv.nib[q >> 3];
            nb_n = rv.nib[(q >> 3) + 1];
            ha_n = rv.hib[q >> 5];
            hb_n = rv.hib[(q >> 5) + 1];
            q_n = q;
        };
        fetch(-u);
        // nothing in flight on loop entry (see packed_sweep)
        __builtin_amdgcn_s_waitcnt(0x0F70);
#pragma unroll 1
        for (int t = 0; t < T; ++t) {
            const int c = t - u;
            const bool act = gact && c >= 0 && c < my_chunks;
            uint4 tc[SW];
#pragma unroll
            for (int w = 0; w < SW; ++w) tc[w] = u == 0 ? tc_n[w] : x_up[w];
            uint32_t nw = __builtin_amdgcn_alignbit(nb_n, na_n, (uint32_t)(q_n & 7) * 4u);
            uint32_t hw = __builtin_amdgcn_alignbit(hb_n, ha_n, (uint32_t)(q_n & 31));
            if (t + 1 < T) fetch(c + 1);
            uint32_t bot[4 * SW];
#pragma unroll
            for (int w = 0; w < 4 * SW; ++w) bot[w] = 0;
            if (act) {
                const int valid = min(N - 8 * c, 8);
                if (valid < 8) {
                    if (REV) {
                        const uint32_t m4 = 0xFFFFFFFFu >> (4 * valid);
                        nw = (nw & ~m4) | (0x88888888u & m4);
                        hw |= 0xFFu >> valid;
                    } else {
                        const uint32_t m4 = 0xFFFFFFFFu << (4 * valid);
                        nw = (nw & ~m4) | (0x88888888u & m4);
                        hw |= (0xFFu << valid) & 0xFFu;
                    }
                }
                uint32_t top[4 * SW];
#pragma unroll
                for (int w = 0; w < SW; ++w) {
                    top[4 * w] = tc[w].x;
                    top[4 * w + 1] = tc[w].y;
                    top[4 * w + 2] = tc[w].z;
                    top[4 * w + 3] = tc[w].w;
                }
                auto code_of = [&](int k) -> uint32_t {
                    const int nb = REV ? 7 - k : k;
                    return ((nw >> (4 * nb)) & 15u) | (((hw >> nb) & 1u) << 4);
                };
                uint32_t w[R / 8];
                load_profile<R>(prof_lane, code_of(0), w);
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    uint32_t wn[R / 8];
                    if (k < 7) load_profile<R>(prof_lane, code_of(k + 1), wn);
                    __builtin_amdgcn_sched_barrier(0);
                    int htop, F;
                    uint32_t tag;
                    if constexpr (WIDE) {
                        htop = (int)top[2 * k];
                        F = (int)top[2 * k + 1];
                        tag = (uint32_t)uni(4095 - ((8 * t + k) & 4095));
                    } else {
                        htop = (int)(top[k] & 0xFFFFu);
                        F = (int)(top[k] >> 16);
                        tag = (uint32_t)uni(0xFFFF - (8 * t + k));
                    }
                    if constexpr (SCAN)
                        column_scan<R>(H, E, mx, w, hdiag, F, go, ge);
                    else
                        column_step<R, TB>(H, E, K, w, hdiag, F, tag, go, ge);
                    hdiag = htop;
                    if constexpr (WIDE) {
                        bot[2 * k] = (uint32_t)H[R - 1];
                        bot[2 * k + 1] = (uint32_t)F;
                    } else {
                        bot[k] = (uint32_t)H[R - 1] | ((uint32_t)F << 16);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    if (k < 7) {
#pragma unroll
                        for (int i = 0; i < R / 8; ++i) w[i] = wn[i];
                    }
                }
            }
            // publish the bottom row of chunk c; lane u+1 reads it at the next
            // step exactly when it processes chunk c, i.e. when this lane was
            // active now
            if constexpr (P > 1) {
#pragma unroll
                for (int w = 0; w < SW; ++w)
                    x_mine[w] = make_uint4(bot[4 * w], bot[4 * w + 1], bot[4 * w + 2], bot[4 * w + 3]);
            }
            if (u == P - 1 && act && write_next) {
#pragma unroll
                for (int w = 0; w < SW; ++w)
                    wr4[c * G * SW + w] = make_uint4(bot[4 * w], bot[4 * w + 1], bot[4 * w + 2], bot[4 * w + 3]);
            }
            if constexpr (WIDE && !SCAN) {
                if ((t & 511) == 511) fold(8 * t + 7 - 4095);
            }
        }
        block_fence();
        if constexpr (SCAN) {
            int gm = mx;
#pragma unroll
            for (int o = 1; o < P; o <<= 1) gm = max(gm, __shfl_xor(gm, o, kWave));
            if (gact) {
                if (REV) {
                    if (gm >= target) {
                        pick = StripPick{gm, sv, bi};
                        done = true;
                    } else {
                        const int tt = bi;
                        bi = bo;
                        bo = tt;
                    }
                } else if (gm > pick.s) {
                    pick = StripPick{gm, sv, bi};
                    const int tt = bk;
                    bk = bi;
                    bi = bo;
                    bo = tt;
                } else {
                    const int tt = bi;
                    bi = bo;
                    bo = tt;
                }
            }
            continue;
        }
        if constexpr (WIDE) {
            fold((8 * T - 1) & ~4095);
        } else if (gact) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int sc = (int)(K[r] >> 16);
                if (row0 + r < M && sc > b.s) {
                    b.s = sc;
                    b.i = row0 + r;
                    b.j = (int)(0xFFFFu - (K[r] & 0xFFFFu)) - 8 * u;
                }
            }
        }
        if (REV) {
            const Best gb = group_best<P>(b);
            if (gact && gb.s >= target) done = true;
        }
    }
    if constexpr (SCAN) {
        if (pick_out) *pick_out = pick;
        return Best{pick.s, -1, -1};
    }
    return group_best<P>(b);
}

// ------------------------------------------------------------------ packed 16-bit score pass
// Groups of P lanes per pair (P = 1, 8 or 16) with 16 rows per lane, two cells
// per 32-bit register: lane u of a group holds rows 16 P ss + 16 u + 0..7
// (half A) in the low 16 bits and rows + 8..15 (half B) in the high 16 bits,
// and B runs one column behind A, so at each step A updates column t and B
// column t - 1 and every packed instruction does two cells of the recurrence.
// As in group_sweep, lane u processes chunk c = t - u at iteration t; its A
// half needs the bottom row of lane u - 1 (from the slot for u = 0), whose
// columns 8c .. 8c+6 were finished in the previous iteration and column
// 8c + 7 in the first step of this one, handed over in the middle of the
// iteration.  Scores carry kScoreBias (pad 0, i.e. -4), the diagonal term is
// sat(Hdiag + s + bias - bias), and E, F and hg saturate at 0 as in the int32
// path, so real cells get the int32 values exactly.  Narrow cells (both
// lengths <= 4096) keep every value below 11 * 4096 + 15 < 2^16.  Padding rows
// and columns only hold values below the pair's maximum, so they cannot change
// the best score or which super-strip first reaches it.
//
// The pass keeps per row a running maximum only.  Forward: the pair's best
// score and the first super-strip that reaches it, whose input boundary row is
// kept by rotating three boundary buffers (one lane per pair: see RING below);
// REV: the first super-strip whose
// maximum reaches `target`, its input row still in the buffer it was read
// from.  group_sweep<ONE> then recomputes that one super-strip in int32 with
// cell trackers.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u16x2 as_u16x2(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t as_u32(u16x2 x) { return __builtin_bit_cast(uint32_t, x); }

// Maximum of three packed cells.  With F16 the 16-bit values are read as
// half-precision bit patterns and one v_pk_maximum3_f16 takes the IEEE
// maximum: for patterns below 0x7C00 (non-negative, finite, subnormals kept
// by the kernels' float mode) the order of the halves is the order of the
// integers, and a maximum only selects one of its inputs, so the result is
// the integer maximum, bit for bit.  Every value a pass holds stays at or
// below its pair's best score, so F16 applies while that bound is below
// kF16MaxScore.
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
constexpr int kF16MaxScore = 31000;
// Largest score a packed pass may hold: every cell stays at or below the
// pair's score and the biased diagonal sum at most 15 above it, all below
// 2^16.
constexpr int kPackedMaxScore = 65504;
// Widest region the narrow recompute tracks: its 16-bit column tags count
// steps of the wavefront (columns plus 8 per lane of offset).
constexpr int kNarrowMaxCols = 65000;
template <bool F16>
__device__ __forceinline__ u16x2 max3_u16x2(u16x2 a, u16x2 b, u16x2 c)
{
    if constexpr (F16) {
        const f16x2 m = __builtin_elementwise_maximum(
            __builtin_elementwise_maximum(__builtin_bit_cast(f16x2, a), __builtin_bit_cast(f16x2, b)),
            __builtin_bit_cast(f16x2, c));
        return __builtin_bit_cast(u16x2, m);
    } else {
        return __builtin_elementwise_max(__builtin_elementwise_max(a, b), c);
    }
}

// Keeps the compiler from moving memory accesses across this point (LDS
// hand-over between lanes of one wave; the hardware keeps a wave's LDS
// accesses in order).
__device__ __forceinline__ void mem_order() { asm volatile("" ::: "memory"); }

// ONE: the exact cells instead of a pick.  Only super-strip `one_ss` (the
// one a score-only pass picked; per group) is swept, from the boundary row in
// buffer `one_buf`, writing nothing; each register keeps, per half (one row),
// the largest (0xFFFF - column) over the cells that reach `target` -- the
// pass's values never exceed it, so sat(H - (target - 1)) is 1 exactly there
// -- which gives every row's first such column, and the group's first row
// with one is the cell the int32 recompute with trackers would report.
template <int P, bool REV, bool F16, bool ONE = false>
__device__ __forceinline__ StripPick packed_sweep(const Args& a, uint8_t* prof, uint32_t* xw, uint32_t* __restrict__ slot,
                                  int64_t Q0, int M, int64_t R0, int N, int target, int one_ss = -1,
                                  int one_buf = 0, Best* one_out = nullptr)
{
    constexpr int G = kWave / P;
    const int64_t BW = narrow_buf_words(P, N);
    const int lane = threadIdx.x & (kWave - 1);
    const int u = lane % P, g = lane / P;
    const uint8_t* prof_lane = prof + lane * prof_bytes(16);
    const unsigned short go16 = (unsigned short)min(a.go, 65535), ge16 = (unsigned short)min(a.ge, 65535);
    const u16x2 go2 = {go16, go16}, ge2 = {ge16, ge16};
    const u16x2 bias2 = {(unsigned short)kScoreBias, (unsigned short)kScoreBias};
    const int my_ss = (M > 0 && N > 0) ? (M + 16 * P - 1) / (16 * P) : 0;
    const int my_chunks = (N + 7) / 8;
    const int wss = uni(wave_max(my_ss));
    const int wc = uni(wave_max(my_ss > 0 ? my_chunks : 0));
    bool done = my_ss == 0 || (REV && target <= 0);
    const bool one_ok = ONE && target > 0 && one_ss >= 0 && one_ss < my_ss;
    const SeqView qv = seq_view(a.qblk, a.qhdr, Q0);
    const SeqView rv = seq_view(a.rblk, a.rhdr, R0);
    uint32_t* grp_slot = slot + 8 * g;  // [buffer][chunk][group][8 cells]
    // hand-over between lanes: 8 words per lane at the end of an iteration
    // (7 used) and one word in the middle
    uint32_t* x_end = xw + 8 * lane;
    const uint32_t* x_end_up = xw + 8 * (lane > 0 ? lane - 1 : 0);
    uint32_t* x_mid = xw + 8 * kWave + lane;
    const uint32_t* x_mid_up = xw + 8 * kWave + (lane > 0 ? lane - 1 : 0);
    int bi = 0, bo = 1, bk = 2;  // boundary buffers: input, output, kept (uniform in a group)
    // One lane per pair: per-lane buffer choices would split each chunk's
    // loads and stores over several buffers, so every lane takes the same
    // ones, in turn: two for the start pass (a pass that stops writes nothing
    // more), a ring of four for the forward pass, whose rows then live for
    // three super-strips.  A lane's best row that outlives the next
    // super-strip is copied during the one after (its source then neither
    // read nor written) to region kKeptBuf, copy loads one chunk ahead.
    constexpr bool RING = P == 1 && !REV && !ONE;
    constexpr int kRingBufs = REV ? 2 : 4;
    bool cp = false, cp_next = false;  // RING: copy row cp_src during this super-strip
    int cp_src = 0;
    StripPick pick{0, -1, 0};
    auto chunk_x = [&](int c) __attribute__((always_inline)) -> int { return (c < 0 || 8 * c >= N) ? 0 : (REV ? -8 * c - 7 : 8 * c); };

    // one lane per pair: the reference's first staged batch is the same for
    // every strip, so it is loaded once and kept in registers
    uint4 b0n0, b0n1, b0n2, b0h0, b0h1;
    if constexpr (P == 1) {
        const int lo0 = REV ? rv.off - 7 - 56 : rv.off;
        const uint4* np = reinterpret_cast<const uint4*>(rv.nib + ((lo0 >> 3) & ~3));
        const uint4* hp = reinterpret_cast<const uint4*>(rv.hib + ((lo0 >> 5) & ~3));
        b0n0 = np[0];
        b0n1 = np[1];
        b0n2 = np[2];
        b0h0 = hp[0];
        b0h1 = hp[1];
    }
    // the query words of the next super-strip are loaded during the current
    // one and decoded when it starts
    uint32_t rq[2][4];
    int rqq[2];
    auto row_raw = [&](int r0) __attribute__((always_inline)) {
        const int x = r0 >= M ? 0 : (REV ? -r0 - 15 : r0);
#pragma unroll
        for (int k8 = 0; k8 < 2; ++k8) {
            const int q = qv.off + x + 8 * k8;
            rq[k8][0] = qv.nib[q >> 3];
            rq[k8][1] = qv.nib[(q >> 3) + 1];
            rq[k8][2] = qv.hib[q >> 5];
            rq[k8][3] = qv.hib[(q >> 5) + 1];
            rqq[k8] = q;
        }
    };
    if constexpr (ONE) row_raw(one_ok ? one_ss * 16 * P + 16 * u : M);
    else row_raw(my_ss > 0 ? 16 * u : M);
    const unsigned short tm1s = (unsigned short)max(target - 1, 0);
    const u16x2 tm1 = {tm1s, tm1s};  // ONE: a cell reaches the target when sat(H - tm1) is 1
    uint32_t Trk[8];                  // ONE: per row, the largest 0xFFFF - column that reaches it
#pragma unroll
    for (int i = 0; i < 8; ++i) Trk[i] = 0;
    if constexpr (ONE) *one_out = Best{0, -1, -1};
#pragma unroll 1
    for (int ss = 0; ss < (ONE ? 1 : wss); ++ss) {
        if (__ballot(ONE ? one_ok : (!done && ss < my_ss)) == 0) break;
        const bool gact = ONE ? one_ok : (!done && ss < my_ss);
        const int sv = ONE ? one_ss : ss;  // super-strip index (per group in ONE)
        const int row0 = sv * 16 * P + 16 * u;
        {
            uint32_t qc[16];
            const int r0 = gact ? row0 : M;
#pragma unroll
            for (int k8 = 0; k8 < 2; ++k8) {
                const uint32_t nw = __builtin_amdgcn_alignbit(rq[k8][1], rq[k8][0], (uint32_t)(rqq[k8] & 7) * 4u);
                const uint32_t hw = __builtin_amdgcn_alignbit(rq[k8][3], rq[k8][2], (uint32_t)(rqq[k8] & 31));
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int idx = 8 * k8 + k;
                    const int r = REV ? (15 - idx) : idx;
                    const uint32_t cd = ((nw >> (4 * k)) & 15u) | (((hw >> k) & 1u) << 4);
                    qc[r] = (r0 + r < M) ? cd : (uint32_t)kPadCode;
                }
            }
            build_profile<16>(prof, lane, qc);
        }
        const bool read_top = sv > 0;
        const bool write_next = !ONE && ss + 1 < my_ss;
        // the first super-strip reads zeros (one 32-byte row for all chunks)
        const int in_buf = ONE ? min(max(one_buf, 0), P == 1 ? kKeptBuf : 2) : bi;
        const uint4* in4 = read_top ? reinterpret_cast<const uint4*>(grp_slot + in_buf * BW) : g_zero_row;
        const int in_stride = read_top ? G * 2 : 0;
        uint4* out4 = reinterpret_cast<uint4*>(grp_slot + bo * BW);
        uint32_t H[8], E[8], Mx[4];  // Mx[k]: running maximum of registers 2k and 2k + 1
#pragma unroll
        for (int i = 0; i < 8; ++i) H[i] = E[i] = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) Mx[i] = 0;
        uint32_t up_prev = 0, fo_prev = 0, pw0 = 0, pw1 = 0;  // previous profile entry
        uint32_t botp[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) botp[k] = 0;
        uint4 tn0 = make_uint4(0, 0, 0, 0), tn1 = make_uint4(0, 0, 0, 0);
        // one lane per pair: the boundary row is loaded two chunks ahead.
        // Iterations go in pairs: the first reads set tn and loads chunks
        // c + 2 into tn and c + 3 into tr, the second reads set tq and then
        // takes tr into tq (by then tr has had two iterations to arrive).
        uint4 tq0 = make_uint4(0, 0, 0, 0), tq1 = make_uint4(0, 0, 0, 0);
        uint4 tr0 = make_uint4(0, 0, 0, 0), tr1 = make_uint4(0, 0, 0, 0);
        uint32_t nw_n = 0, hw_n = 0;
        // RING: the chunks of the copy in flight (even chunks in set n, odd
        // in set q: a load never takes the registers a store just read), its
        // source and destination
        uint4 cn0 = make_uint4(0, 0, 0, 0), cn1 = make_uint4(0, 0, 0, 0);
        uint4 cq0 = make_uint4(0, 0, 0, 0), cq1 = make_uint4(0, 0, 0, 0);
        bool any_cp = false;
        if constexpr (RING) any_cp = __ballot(cp) != 0;
        const uint4* cp4 = reinterpret_cast<const uint4*>(grp_slot + (int64_t)cp_src * BW);
        uint4* kept4 = reinterpret_cast<uint4*>(grp_slot + (int64_t)kKeptBuf * BW);
        // One lane per pair: the reference comes through LDS.  Every 8 chunks
        // a lane loads the aligned 16-byte groups holding the next 72
        // residues (3 of the nibble plane, 2 of the high plane) one batch
        // ahead and writes them to its column of the staging area ([word]
        // [lane], conflict-free for any per-lane offset); each chunk reads
        // its two words per plane from there.  Per-chunk global loads of
        // scattered words missed the L1 most of the time.
        uint4 sn0, sn1, sn2, sh0, sh1;  // staged batch
        const int s0 = rv.off + (REV ? -7 : 0);
        const int last_batch = max(my_chunks - 1, 0) >> 3;
        auto batch_lo = [&](int bb) __attribute__((always_inline)) -> int {
            const int b = min(bb, last_batch);  // lanes past their end re-read their last batch
            return REV ? s0 - 64 * b - 56 : s0 + 64 * b;
        };
        auto load_batch = [&](int bb) __attribute__((always_inline)) {
            const int lo = batch_lo(bb);
            const uint4* np = reinterpret_cast<const uint4*>(rv.nib + ((lo >> 3) & ~3));
            const uint4* hp = reinterpret_cast<const uint4*>(rv.hib + ((lo >> 5) & ~3));
            sn0 = np[0];
            sn1 = np[1];
            sn2 = np[2];
            sh0 = hp[0];
            sh1 = hp[1];
        };
        auto store_batch = [&]() __attribute__((always_inline)) {
            const uint32_t v[20] = {sn0.x, sn0.y, sn0.z, sn0.w, sn1.x, sn1.y, sn1.z, sn1.w, sn2.x, sn2.y,
                                    sn2.z, sn2.w, sh0.x, sh0.y, sh0.z, sh0.w, sh1.x, sh1.y, sh1.z, sh1.w};
#pragma unroll
            for (int w = 0; w < 20; ++w) xw[w * kWave + lane] = v[w];
        };
        // window of chunk c from the staged batch c / 8
        auto window_lds = [&](int c) __attribute__((always_inline)) {
            const int b = c >> 3, j = c & 7;
            const int lo = batch_lo(b);
            const int st = REV ? lo + 56 - 8 * j : lo + 8 * j;  // first residue of the window
            // inside the staged words (lanes past their end re-read their last batch)
            const int wn = min((st >> 3) - ((lo >> 3) & ~3), 10);
            const int wh = min((st >> 5) - ((lo >> 5) & ~3), 6);
            const uint32_t n0 = xw[wn * kWave + lane], n1 = xw[(wn + 1) * kWave + lane];
            const uint32_t h0 = xw[(12 + wh) * kWave + lane], h1 = xw[(13 + wh) * kWave + lane];
            nw_n = __builtin_amdgcn_alignbit(n1, n0, (uint32_t)(st & 7) * 4u);
            hw_n = __builtin_amdgcn_alignbit(h1, h0, (uint32_t)(st & 31));
        };
        auto fetch = [&](int cn) __attribute__((always_inline)) {
            // an index inside the pair's chunks: the columns past the last
            // chunk (padding, scored -4 against everything) get the last
            // chunk's boundary, real cells of the row above, so their values
            // stay below the pair's maximum.  Lanes u > 0 take their top
            // row from lane u - 1 instead.
            const int cc = min(max(cn, 0), max(my_chunks - 1, 0));
            tn0 = in4[cc * in_stride];
            tn1 = in4[cc * in_stride + 1];
            if constexpr (P > 1) window8(rv, chunk_x(cn), nw_n, hw_n);
        };
        auto fetch_q = [&](int cn) __attribute__((always_inline)) {
            const int cc = min(max(cn, 0), max(my_chunks - 1, 0));
            tq0 = in4[cc * in_stride];
            tq1 = in4[cc * in_stride + 1];
        };
        auto fetch_r = [&](int cn) __attribute__((always_inline)) {
            const int cc = min(max(cn, 0), max(my_chunks - 1, 0));
            tr0 = in4[cc * in_stride];
            tr1 = in4[cc * in_stride + 1];
        };
        fetch(-u);
        if constexpr (P == 1) fetch_q(1);
        if constexpr (P == 1) {
            sn0 = b0n0;
            sn1 = b0n1;
            sn2 = b0n2;
            sh0 = b0h0;
            sh1 = b0h1;
            store_batch();
        }
        // Nothing in flight when the chunk loop starts: a load still pending
        // on entry makes the compiler keep waits for it inside the loop,
        // which then stall on the loads issued in the same iteration.
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt and lgkmcnt untouched
        if constexpr (P == 1) {
            load_batch(1);
            window_lds(0);
        }
        if constexpr (!ONE) row_raw(ss + 1 < my_ss ? row0 + 16 * P : M);
        // Iteration t: lane u on chunk c = t - u, A on columns 8c .. 8c+7,
        // B on 8c-1 .. 8c+6.  Each lane needs my_chunks + 1 chunk iterations
        // (the last one for B's final column); the very last iteration of the
        // wave has a single step.
        // With one lane per pair, iteration t reads its row from set tn (t
        // even) or tq (t odd).
        auto iteration = [&](int t, auto steps_tag, auto set_tag) __attribute__((always_inline)) {
            constexpr int STEPS = decltype(steps_tag)::value;
            constexpr bool SET_Q = P == 1 && decltype(set_tag)::value;
            const int c = t - u;
            const bool act = gact && c >= 0 && c <= my_chunks;
            const int tag0 = 0xFFFF - 8 * c;  // ONE: tag of column 8c (A); B is one column behind
            uint32_t top[8];
            if constexpr (SET_Q) {
                top[0] = tq0.x, top[1] = tq0.y, top[2] = tq0.z, top[3] = tq0.w;
                top[4] = tq1.x, top[5] = tq1.y, top[6] = tq1.z, top[7] = tq1.w;
            } else {
                top[0] = tn0.x, top[1] = tn0.y, top[2] = tn0.z, top[3] = tn0.w;
                top[4] = tn1.x, top[5] = tn1.y, top[6] = tn1.z, top[7] = tn1.w;
            }
            if constexpr (P == 1) {
                // copies of their own, so that the set's registers take the
                // next load at once and keep them across the loop
#pragma unroll
                for (int k = 0; k < 8; ++k) opaque(top[k]);
                __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (RING) {
                // the copy: chunk c - 1 (loaded one iteration ago, before
                // that iteration's boundary loads, so waiting for it waits
                // for nothing younger), then the load of chunk c
                if (any_cp) {
                    if (cp && c >= 1 && c - 1 < my_chunks) {
                        kept4[(c - 1) * (G * 2)] = SET_Q ? cn0 : cq0;
                        kept4[(c - 1) * (G * 2) + 1] = SET_Q ? cn1 : cq1;
                    }
                    if (cp && c < my_chunks) {
                        if constexpr (SET_Q) {
                            cq0 = cp4[c * (G * 2)];
                            cq1 = cp4[c * (G * 2) + 1];
                        } else {
                            cn0 = cp4[c * (G * 2)];
                            cn1 = cp4[c * (G * 2) + 1];
                        }
                    }
                }
            }
            if constexpr (P > 1) {
                // both sources are read and the values selected (a select of
                // addresses would turn into flat loads)
                const uint4 e0 = reinterpret_cast<const uint4*>(x_end_up)[0];
                const uint4 e1 = reinterpret_cast<const uint4*>(x_end_up)[1];
                const bool up = u > 0;
                top[0] = up ? e0.x : top[0];
                top[1] = up ? e0.y : top[1];
                top[2] = up ? e0.z : top[2];
                top[3] = up ? e0.w : top[3];
                top[4] = up ? e1.x : top[4];
                top[5] = up ? e1.y : top[5];
                top[6] = up ? e1.z : top[6];
            }
            uint32_t nw = nw_n, hw = hw_n;
            if constexpr (P == 1) {
                // c == t here.  The next chunk's window is read now (from the
                // next batch when one starts there: staged data to LDS first,
                // the batch after it in flight).
                if ((c & 7) == 7) {
                    store_batch();
                    load_batch((c >> 3) + 2);
                }
                window_lds(c + 1);
            }
            if constexpr (P == 1) {
                // unconditional (the index is clamped), so that each set
                // keeps its registers from one pair of iterations to the next
                if constexpr (!SET_Q) {
                    fetch(c + 2);
                    fetch_r(c + 3);
                }
            } else if (t + 1 <= wc + P - 1) {
                fetch(c + 1);
            }
            // B's row 15 per step.  An idle lane hands zeros to lane u + 1;
            // with one lane per pair the values are only read after an
            // active iteration, so nothing is cleared.
            uint32_t bq[8];
            if constexpr (P > 1) {
#pragma unroll
                for (int k = 0; k < 8; ++k) bq[k] = 0;
            }
            const int valid = min(max(N - 8 * c, 0), 8);
            if (valid < 8) {
                if (REV) {
                    const uint32_t m4 = valid == 0 ? 0xFFFFFFFFu : (0xFFFFFFFFu >> (4 * valid));
                    nw = (nw & ~m4) | (0x88888888u & m4);
                    hw |= 0xFFu >> valid;
                } else {
                    const uint32_t m4 = 0xFFFFFFFFu << (4 * valid);
                    nw = (nw & ~m4) | (0x88888888u & m4);
                    hw |= (0xFFu << valid) & 0xFFu;
                }
            }
            auto code_of = [&](int k) __attribute__((always_inline)) -> uint32_t {
                const int nb = REV ? 7 - k : k;
                return ((nw >> (4 * nb)) & 15u) | (((hw >> nb) & 1u) << 4);
            };
            uint32_t w[2], wn[2];
            // one step: A on column 8c + k, B on column 8c + k - 1
            auto step = [&](int k) __attribute__((always_inline)) {
                if (k + 1 < STEPS) load_profile<16>(prof_lane, code_of(k + 1), wn);
                // low halves from this column's entry (A rows), high halves
                // from the previous one (B rows): register i gets nibble i & 3
                // of both
                // (one v_bfi each; opaque keeps the masks below from being
                // folded into it, which costs two more instructions)
                uint32_t x0 = (pw0 & 0xFFFF0000u) | (w[0] & 0xFFFFu);
                uint32_t x1 = (pw1 & 0xFFFF0000u) | (w[1] & 0xFFFFu);
                opaque(x0);
                opaque(x1);
                uint32_t sw[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint32_t x = i < 4 ? x0 : x1;
                    if ((i & 3) == 3) {  // the top nibble of each half: one packed shift
                        const u16x2 t12 = {12, 12};
                        sw[i] = as_u32(as_u16x2(x) >> t12);
                    } else {
                        sw[i] = (x >> (4 * (i & 3))) & 0x000F000Fu;
                    }
                }
                // row 0 inputs: A from the row above at column t, B from A's
                // row 7 at column t - 1
                const uint32_t up_cur = __builtin_amdgcn_perm(H[7], top[k], 0x05040100u);
                uint32_t Fv = __builtin_amdgcn_perm(fo_prev, top[k], 0x05040302u);
                uint32_t hd = up_prev;
                u16x2 h_even = {0, 0};
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    // saturating: a value beyond 16 bits stays at 65535 (a pass
                    // that reaches it gives up, see the strip maximum below)
                    const u16x2 d = __builtin_elementwise_sub_sat(
                        __builtin_elementwise_add_sat(as_u16x2(hd), as_u16x2(sw[i])), bias2);
                    const u16x2 h = max3_u16x2<F16>(d, as_u16x2(E[i]), as_u16x2(Fv));
                    hd = H[i];
                    H[i] = as_u32(h);
                    const u16x2 hg = __builtin_elementwise_sub_sat(h, go2);
                    E[i] = as_u32(__builtin_elementwise_max(__builtin_elementwise_sub_sat(as_u16x2(E[i]), ge2), hg));
                    Fv = as_u32(__builtin_elementwise_max(__builtin_elementwise_sub_sat(as_u16x2(Fv), ge2), hg));
                    if constexpr (!ONE) {
                        if (i & 1) Mx[i / 2] = as_u32(max3_u16x2<F16>(as_u16x2(Mx[i / 2]), h_even, h));
                        else h_even = h;
                    }
                }
                if constexpr (ONE) {
                    const u16x2 tg = {(unsigned short)(tag0 - k), (unsigned short)(tag0 - k + 1)};
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        Trk[i] = as_u32(__builtin_elementwise_max(
                            as_u16x2(Trk[i]), __builtin_elementwise_sub_sat(as_u16x2(H[i]), tm1) * tg));
                }
                fo_prev = Fv;
                up_prev = up_cur;
                // B's row 15 at column t - 1 as (H | F << 16)
                bq[k] = __builtin_amdgcn_perm(Fv, H[7], 0x07060302u);
                pw0 = w[0];
                pw1 = w[1];
                w[0] = wn[0];
                w[1] = wn[1];
            };
            if (act) {
                load_profile<16>(prof_lane, code_of(0), w);
                step(0);
            }
            if (P > 1) {
                *x_mid = bq[0];  // column 8c - 1, for lane u + 1's chunk c - 1
                mem_order();
            }
            // chunk c-1 of the bottom row is complete: columns 8c-8 .. 8c-2
            // from the previous iteration, 8c-1 from this one's first step.
            // Stored here, early: stores and loads share one counter, so a
            // store still in flight at the end of the iteration would hold
            // up the wait for the next chunk's loads.  (Whole 32-byte rows:
            // split partial stores measured slower.)
            if (u == P - 1 && act && write_next && c >= 1 && c - 1 < my_chunks) {
                out4[(c - 1) * (G * 2)] = make_uint4(botp[1], botp[2], botp[3], botp[4]);
                out4[(c - 1) * (G * 2) + 1] = make_uint4(botp[5], botp[6], botp[7], bq[0]);
            }
            if (act) {
#pragma unroll
                for (int k = 1; k < STEPS; ++k) {
                    if (P > 1 && k == 7) {
                        // column 8c + 7 of the row above, finished by lane
                        // u - 1 in its first step of this iteration
                        const uint32_t xm = *x_mid_up;
                        top[7] = u > 0 ? xm : top[7];
                    }
                    step(k);
                }
            }
            if (P > 1) {
                // columns 8c .. 8c+6 for lane u + 1's next iteration
                mem_order();
                reinterpret_cast<uint4*>(x_end)[0] = make_uint4(bq[1], bq[2], bq[3], bq[4]);
                reinterpret_cast<uint4*>(x_end)[1] = make_uint4(bq[5], bq[6], bq[7], 0u);
                mem_order();
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) botp[k] = bq[k];
            if constexpr (SET_Q) {
                tq0 = tr0;
                tq1 = tr1;
            }
        };
        const int T = wc + P;  // iterations 0 .. wc + P - 1
        using Full = std::integral_constant<int, 8>;
        using Last = std::integral_constant<int, 1>;
        using SetN = std::integral_constant<bool, false>;
        using SetQ = std::integral_constant<bool, true>;
        if constexpr (P == 1) {
            // iterations in pairs (sets tn, tq), then what is left: the
            // last full one (set tn) if T is even, and the last (one step)
            int t = 0;
#pragma unroll 1
            for (; t + 1 < T - 1; t += 2) {
                iteration(t, Full(), SetN());
                iteration(t + 1, Full(), SetQ());
            }
            if (t < T - 1) {
                iteration(t, Full(), SetN());
                iteration(T - 1, Last(), SetQ());
            } else {
                iteration(T - 1, Last(), SetN());
            }
        } else {
#pragma unroll 1
            for (int t = 0; t < T - 1; ++t) iteration(t, Full(), SetN());
            iteration(T - 1, Last(), SetN());
        }
        block_fence();
        if constexpr (ONE) {
            // the lane's first row with a cell at the target, then the
            // group's first (rows 0-7 in the low halves, 8-15 in the high)
            Best b{0, -1, -1};
            if (gact) {
#pragma unroll
                for (int r = 15; r >= 0; --r) {
                    const uint32_t v = r < 8 ? (Trk[r] & 0xFFFFu) : (Trk[r - 8] >> 16);
                    if (v != 0 && row0 + r < M) b = Best{target, row0 + r, 0xFFFF - (int)v};
                }
            }
            *one_out = group_best<P>(b);
            return pick;
        }
        uint32_t m2 = Mx[0];
#pragma unroll
        for (int i = 1; i < 4; ++i) m2 = as_u32(__builtin_elementwise_max(as_u16x2(m2), as_u16x2(Mx[i])));
        int smax = (int)max(m2 & 0xFFFFu, m2 >> 16);
#pragma unroll
        for (int o = 1; o < P; o <<= 1) smax = max(smax, __shfl_xor(smax, o, kWave));
        if (gact) {
            if (P == kWave && !F16 && smax > kPackedMaxScore) {
                // some value may not fit 16 bits: the pair continues in int32
                // from this super-strip, whose input row (every value of the
                // super-strips above is exact) stays in buffer bi.  (Only a
                // whole wave gets pairs long enough; half-precision passes
                // run only under kF16MaxScore.)
                pick.s = -1;
                pick.ss = ss;
                pick.buf = bi;
                done = true;
            } else if (REV) {
                if (smax >= target) {
                    pick.ss = ss;
                    pick.buf = bi;
                    done = true;
                } else if (P > 1) {
                    const int tt = bi;
                    bi = bo;
                    bo = tt;
                }
            } else if (RING) {
                if (smax > pick.s) {
                    pick.s = smax;
                    pick.ss = ss;
                    pick.buf = bi;
                } else {
                    // the copy made during this super-strip now holds the
                    // best row; a best row one super-strip old that the
                    // ring would overwrite is copied during the next one
                    if (cp) pick.buf = kKeptBuf;
                    cp_next = pick.ss == ss - 1 && pick.ss > 0 && pick.ss + kRingBufs < my_ss;
                    cp_src = pick.buf;
                }
            } else if (smax > pick.s) {
                pick.s = smax;
                pick.ss = ss;
                pick.buf = bi;
                const int tt = bk;
                bk = bi;
                bi = bo;
                bo = tt;
            } else {
                const int tt = bi;
                bi = bo;
                bo = tt;
            }
        }
        if constexpr (P == 1) {
            // the same buffers on every lane, finished or not (a finished
            // lane writes nothing, and a row it keeps is named by its pick)
            bi = bo;
            bo = bo + 1 == kRingBufs ? 0 : bo + 1;
            cp = cp_next;
            cp_next = false;
        }
    }
    return pick;
}

// ------------------------------------------------------------------ work cells
__device__ __forceinline__ int ceil_log2(int64_t x)
{
    int b = 0;
    while (((int64_t)1 << b) < x) ++b;
    return b;
}

// Lanes per pair of a work cell: 1 for the short-pair cells; for long pairs
// by length bucket 8 up to group8_max, 16 up to group16_max (both at most
// kMaxP16Len residues), 64 beyond.
__device__ __forceinline__ int cell_kind(int cell, const Args& a)
{
    if (cell < kInterCells) return 1;
    const int bucket = (cell - kInterCells) / kWideCostBins;
    return bucket_group_kind(bucket, a.bucket_kind[bucket], a.group8_max_len, a.group16_max_len);
}

// Cell of a pair of lengths m, n > 0: lane-per-pair pairs by (strips,
// chunks), longer pairs by (length bucket, 16*log2(m*n)).
__device__ __forceinline__ int cell_of(const Args& a, int64_t m, int64_t n)
{
    const int64_t mx = m > n ? m : n;
    const int ov = a.bucket_kind[ceil_log2(mx)];
    if (ov == 1 || (ov == 0 && mx <= a.inter_max_len)) {
        const int s = (int)((m + a.rows_per_lane - 1) / a.rows_per_lane);
        const int c = (int)((n + 7) / 8);
        return (s - 1) * kMaxInterChunks + (c - 1);
    }
    const int64_t cost = m * n;
    const int msb = 63 - __clzll((unsigned long long)cost);
    const int frac = msb >= 4 ? (int)((cost >> (msb - 4)) & 15) : 0;
    const int cb = min(kWideCostBins - 1, 16 * msb + frac);
    return kInterCells + ceil_log2(mx) * kWideCostBins + cb;
}

// Whole wave: copy the narrow boundary row in buffer `nbuf` (one word per
// column, H | F << 16) into a wide buffer of the same slot (two words per
// column, H then F), for an int32 scan to continue from.  The wide buffer is
// the first of the three whose words do not overlap the narrow one's (a wide
// buffer is at least as long, so the narrow one meets at most two); returns
// its index.  Not inlined: the copy runs once per pair that overflows, and
// inlined its registers pushed the persistent kernel into spilling.
__device__ __attribute__((noinline)) int widen_row(uint32_t* __restrict__ slot, int nbuf, int N)
{
    const int64_t BW = narrow_buf_words(kWave, N), WBW = wide_buf_words(N);
    const int64_t lo = (int64_t)nbuf * BW, hi = lo + BW;
    int k = 0;
    while (k < 2 && (int64_t)k * WBW < hi && lo < (int64_t)(k + 1) * WBW) ++k;
    const uint4* src = reinterpret_cast<const uint4*>(slot + lo);
    uint4* dst = reinterpret_cast<uint4*>(slot + (int64_t)k * WBW);
    const int lane = threadIdx.x & (kWave - 1);
    const int chunks = (N + 7) / 8;
#pragma unroll 1
    for (int c = lane; c < chunks; c += kWave) {
        const uint4 a0 = src[2 * c], a1 = src[2 * c + 1];
        const uint32_t v[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
            dst[4 * c + q] = make_uint4(v[2 * q] & 0xFFFFu, v[2 * q] >> 16, v[2 * q + 1] & 0xFFFFu, v[2 * q + 1] >> 16);
    }
    block_fence();
    return k;
}

// ------------------------------------------------------------------ per-item drivers
__device__ __forceinline__ void write_result(sw_result* out, int pid, int S, int qs, int qe, int rs, int re)
{
    sw_result r;
    if (S > 0) {
        r.score = S;
        r.q_start = qs;
        r.q_end = qe;
        r.r_start = rs;
        r.r_end = re;
    } else {
        r.score = 0;
        r.q_start = r.q_end = r.r_start = r.r_end = -1;
    }
    out[pid] = r;
}

// One work item: up to 64/P pairs, P lanes each.  a.phase 0 runs the forward
// pass and the start pass of each pair; phase 1 only the forward pass (score
// and end written, starts -1); phase 2 only the start pass of pairs whose
// score and end are already in `out` (the item then groups pairs by the size
// of their start-pass region, so its lanes finish together).
template <int R, int P, bool WIDE>
__device__ __forceinline__ void do_group(const Args& a, int first, int count, uint8_t* lds, uint32_t* slot)
{
    constexpr int G = kWave / P;
    constexpr int SW = WIDE ? 4 : 2;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / P, u = lane % P;
    int pid = -1, m = 0, n = 0;
    int64_t qoff = 0, roff = 0;
    Best f{0, -1, -1};  // forward result (read back in phase 2)
    if (g < count) {
        pid = a.perm[first + g];
        if (pid < 0 || pid >= a.n_pairs) pid = -1;
    }
    if (pid >= 0) {
        const int qi = a.pairs[2 * pid], ri = a.pairs[2 * pid + 1];
        qoff = a.q_offsets[qi];
        m = (int)(a.q_offsets[qi + 1] - qoff);
        roff = a.r_offsets[ri];
        n = (int)(a.r_offsets[ri + 1] - roff);
        if (a.phase == 2) {
            // the start pass covers q[0..q_end] x r[0..r_end]
            const sw_result r = a.out[pid];
            if (r.score > 0 && r.q_end >= 0 && r.q_end < m && r.r_end >= 0 && r.r_end < n) {
                f = Best{r.score, r.q_end, r.r_end};
                m = r.q_end + 1;
                n = r.r_end + 1;
            } else {
                pid = -1;
                m = n = 0;
            }
        }
    }
    if (pid >= 0) {
        // the slot must hold one boundary cell per column for every group
        // (narrow groups: buffers of fixed size, five for one lane, three
        // for 8 and 16)
        const int64_t need = (int64_t)((n + 7) / 8) * G * SW * 4;
        const bool may_pack = R == 16 && (P == 64 ? max(m, n) <= kMaxP16Len : !WIDE);
        const int max_chunks = P == 1 ? kMaxInterChunks : kMaxP16Len / 8;
        if (need > a.slot_words ||
            (may_pack && ((n + 7) / 8 > max_chunks ||
                          (P == 1 ? kKeptBuf + 1 : 3) * boundary_buf_words(P) > a.slot_words))) {
            if (u == 0) {
                atomicOr((unsigned*)a.err, (unsigned)kErrInternal);
                sw_result bad;
                bad.score = bad.q_start = bad.q_end = bad.r_start = bad.r_end = -1;
                a.out[pid] = bad;
            }
            pid = -1;
            m = n = 0;
            f = Best{0, -1, -1};
        }
    }
    uint8_t* prof = lds;
    uint4* xbuf = reinterpret_cast<uint4*>(lds + kNumCodes * kWave * prof_bytes(R));
    // forward pass done: phase 1 stores score and end, the start pass follows
    // in phase 0
    // in phase 0
    auto forward_done = [&](int packed_s) __attribute__((always_inline)) {
        if (pid >= 0 && u == 0 && packed_s >= 0 && f.s != packed_s)
            atomicOr((unsigned*)a.err, (unsigned)kErrInternal);
        if (a.phase == 1 && pid >= 0 && u == 0) {
            sw_result r;
            r.score = f.s;
            r.q_start = r.r_start = -1;
            r.q_end = f.s > 0 ? f.i : -1;
            r.r_end = f.s > 0 ? f.j : -1;
            a.out[pid] = r;
        }
    };
    // packed score passes for every pair up to kMaxP16Len residues (the one-,
    // 8- and 16-lane groups only get such pairs; a whole wave takes the longest
    // of them and everything beyond, which runs in int32 throughout), then the
    // exact cells from one int32 super-strip each
    bool packed = false;
    if constexpr (R == 16) {
        if constexpr (P == 64) packed = uni(max(m, n)) <= kMaxP16Len;  // one pair per item
        else packed = !WIDE;
    }
    if (packed) {
        uint32_t* xw = reinterpret_cast<uint32_t*>(xbuf);
        if (a.phase != 2) {
            // every value of the forward pass is at most 11 min(m, n)
            const bool f16 = P == 1 || uni(wave_max(11 * min(m, n))) <= kF16MaxScore;
            const StripPick pf = f16 ? packed_sweep<P, false, true>(a, prof, xw, slot, qoff, m, roff, n, 0)
                                     : packed_sweep<P, false, false>(a, prof, xw, slot, qoff, m, roff, n, 0);
            // the first cell of the best score, in the super-strip picked
            if (f16)
                packed_sweep<P, false, true, true>(a, prof, xw, slot, qoff, m, roff, n, pf.s, pf.ss, pf.buf, &f);
            else
                packed_sweep<P, false, false, true>(a, prof, xw, slot, qoff, m, roff, n, pf.s, pf.ss, pf.buf, &f);
            forward_done(pf.s);
            if (a.phase == 1) return;
        }
        const bool hs = f.s > 0;
        const int64_t qr = qoff + (hs ? f.i : 0), rr = roff + (hs ? f.j : 0);
        const int mr = hs ? f.i + 1 : 0, nr = hs ? f.j + 1 : 0;
        // and every value of the start pass at most the score
        const bool f16 = P == 1 || uni(wave_max(f.s)) <= kF16MaxScore;
        const StripPick pr = f16 ? packed_sweep<P, true, true>(a, prof, xw, slot, qr, mr, rr, nr, f.s)
                                 : packed_sweep<P, true, false>(a, prof, xw, slot, qr, mr, rr, nr, f.s);
        Best r{0, -1, -1};
        if (f16)
            packed_sweep<P, true, true, true>(a, prof, xw, slot, qr, mr, rr, nr, f.s, hs ? pr.ss : -1, pr.buf, &r);
        else
            packed_sweep<P, true, false, true>(a, prof, xw, slot, qr, mr, rr, nr, f.s, hs ? pr.ss : -1, pr.buf, &r);
        if (pid >= 0 && u == 0) {
            if (hs && r.s != f.s) atomicOr((unsigned*)a.err, (unsigned)kErrInternal);
            write_result(a.out, pid, f.s, f.i - r.i, f.i, f.j - r.j, f.j);
        }
        return;
    }
    // whole wave, pairs beyond kMaxP16Len.  Forward: a packed pass first (its
    // additions saturate, so any value beyond 16 bits shows as a strip
    // maximum above kPackedMaxScore and the pass stops there), then the
    // exact cells from the packed super-strip.  A pass that stopped goes on
    // as an int32 scan from the super-strip where it stopped (its input row
    // widened), keeping only each super-strip's maximum, then the exact cells
    // from one super-strip with trackers -- when three int32 boundary
    // buffers of the pair fit the slot (the least slot: pairs up to ~54k
    // columns; the library's slots: every pair); else the
    // in-place sweep with trackers in every cell, from the top.  The start
    // pass the same way, packed when the score fits.
    if constexpr (WIDE) {
        const bool scan_fits = 3 * wide_buf_words(n) <= a.slot_words;
        const bool narrow_ok = R == 16 && uni(n) <= kNarrowMaxCols;  // three narrow buffers always fit
        if (a.phase != 2) {
            bool fwd = false;
            int ss0 = 0, buf0 = 0;  // where an int32 scan starts
            if constexpr (R == 16) {
                if (narrow_ok) {
                    uint32_t* xw = reinterpret_cast<uint32_t*>(xbuf);
                    const StripPick pf = packed_sweep<P, false, false>(a, prof, xw, slot, qoff, m, roff, n, 0);
                    if (uni(pf.s) >= 0) {
                        packed_sweep<P, false, false, true>(a, prof, xw, slot, qoff, m, roff, n, pf.s, pf.ss,
                                                            pf.buf, &f);
                        forward_done(pf.s);
                        fwd = true;
                    } else if (scan_fits && uni(pf.ss) > 0) {
                        // every super-strip above pf.ss stayed below
                        // kPackedMaxScore, so the best score (above it) is
                        // reached below: the scan goes on from pf.ss
                        ss0 = uni(pf.ss);
                        buf0 = widen_row(slot, uni(pf.buf), n);
                    }
                }
            }
            if (!fwd && scan_fits) {
                StripPick pf{0, -1, 0};
                group_sweep<R, P, false, true, false, true>(a, prof, xbuf, slot, qoff, m, roff, n, 0, -1, 0, &pf,
                                                            ss0, buf0);
                f = group_sweep<R, P, false, true, true>(a, prof, xbuf, slot, qoff, m, roff, n, 0, pf.ss, pf.buf);
                forward_done(pf.s);
                fwd = true;
            }
            if (!fwd) {
                f = group_sweep<R, P, false, WIDE>(a, prof, xbuf, slot, qoff, m, roff, n, 0);
                forward_done(-1);
            }
            if (a.phase == 1) return;
        }
        const bool hs = f.s > 0;
        const int64_t qr = qoff + (hs ? f.i : 0), rr = roff + (hs ? f.j : 0);
        const int mr = hs ? f.i + 1 : 0, nr = hs ? f.j + 1 : 0;
        Best r{0, -1, -1};
        // Every value of the start pass is at most the score.  The pass runs
        // in packed cells (half-precision maxima when the score is at most
        // kF16MaxScore) and its recompute in narrow cells whose 16-bit column
        // tags cover the region's columns; a score above kPackedMaxScore
        // makes the packed pass stop at the first super-strip whose values
        // pass 16 bits, and the int32 scan goes on from there.
        const bool scan_fits_r = 3 * wide_buf_words(nr) <= a.slot_words;
        bool start_done = false;
        int ss0 = 0, buf0 = 0;  // where an int32 scan starts
        if constexpr (R == 16) {
            if (uni(nr) <= kNarrowMaxCols) {
                uint32_t* xw = reinterpret_cast<uint32_t*>(xbuf);
                if (uni(f.s) <= kF16MaxScore) {
                    const StripPick pr = packed_sweep<P, true, true>(a, prof, xw, slot, qr, mr, rr, nr, f.s);
                    packed_sweep<P, true, true, true>(a, prof, xw, slot, qr, mr, rr, nr, f.s, hs ? pr.ss : -1,
                                                      pr.buf, &r);
                    start_done = true;
                } else {
                    const StripPick pr = packed_sweep<P, true, false>(a, prof, xw, slot, qr, mr, rr, nr, f.s);
                    if (uni(pr.s) >= 0) {
                        packed_sweep<P, true, false, true>(a, prof, xw, slot, qr, mr, rr, nr, f.s,
                                                           hs ? pr.ss : -1, pr.buf, &r);
                        start_done = true;
                    } else if (scan_fits_r && uni(pr.ss) > 0) {
                        // the super-strips above pr.ss stayed below the score
                        ss0 = uni(pr.ss);
                        buf0 = widen_row(slot, uni(pr.buf), nr);
                    }
                }
            }
        }
        if (start_done) {
        } else if (scan_fits_r) {
            StripPick pr{0, -1, 0};
            group_sweep<R, P, true, true, false, true>(a, prof, xbuf, slot, qr, mr, rr, nr, f.s, -1, 0, &pr, ss0,
                                                       buf0);
            r = group_sweep<R, P, true, true, true>(a, prof, xbuf, slot, qr, mr, rr, nr, f.s, hs ? pr.ss : -1,
                                                    pr.buf);
        } else {
            r = group_sweep<R, P, true, WIDE>(a, prof, xbuf, slot, qr, mr, rr, nr, f.s);
        }
        if (pid >= 0 && u == 0) {
            if (hs && r.s != f.s) atomicOr((unsigned*)a.err, (unsigned)kErrInternal);
            write_result(a.out, pid, f.s, f.i - r.i, f.i, f.j - r.j, f.j);
        }
        return;
    }
    if (a.phase != 2) {
        f = group_sweep<R, P, false, WIDE>(a, prof, xbuf, slot, qoff, m, roff, n, 0);
        forward_done(-1);
        if (a.phase == 1) return;
    }
    const bool hs = f.s > 0;
    const Best r = group_sweep<R, P, true, WIDE>(a, prof, xbuf, slot, qoff + (hs ? f.i : 0), hs ? f.i + 1 : 0,
                                                 roff + (hs ? f.j : 0), hs ? f.j + 1 : 0, f.s);
    if (pid >= 0 && u == 0) {
        if (hs && r.s != f.s) atomicOr((unsigned*)a.err, (unsigned)kErrInternal);
        write_result(a.out, pid, f.s, f.i - r.i, f.i, f.j - r.j, f.j);
    }
}

// ------------------------------------------------------------------ kernels
// Work items, in queue order: single pairs over 64 lanes (longest first),
// groups of 4 pairs over 16 lanes each, of 8 pairs over 8 lanes each, of 64
// pairs one per lane.
template <int R>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2))) void k_persistent(Args a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    uint32_t* slot = a.scratch + (int64_t)blockIdx.x * a.slot_words;
    // the counters come from the scan; clamp them so that a bookkeeping error
    // can never index past the permutation
    const int n64 = min(max(a.counters[kCntP64], 0), (int)a.n_pairs);
    const int n16 = min(max(a.counters[kCntP16], 0), (int)a.n_pairs - n64);
    const int n8 = min(max(a.counters[kCntP8], 0), (int)a.n_pairs - n64 - n16);
    const int n1 = min(max(a.counters[kCntP1], 0), (int)a.n_pairs - n64 - n16 - n8);
    const int i16 = (n16 + 3) / 4, i8 = (n8 + 7) / 8, i1 = (n1 + kWave - 1) / kWave;
    const int total = n64 + i16 + i8 + i1;
#pragma unroll 1
    for (;;) {
        int item = 0;
        if ((threadIdx.x & (kWave - 1)) == 0) item = atomicAdd(&a.counters[kCntHead], 1);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= total) break;
        if (item < n64) {
            do_group<R, 64, true>(a, item, 1, lds, slot);
        } else if (item < n64 + i16) {
            const int k = item - n64;
            do_group<R, 16, false>(a, n64 + 4 * k, min(4, n16 - 4 * k), lds, slot);
        } else if (item < n64 + i16 + i8) {
            const int k = item - n64 - i16;
            do_group<R, 8, false>(a, n64 + n16 + 8 * k, min(8, n8 - 8 * k), lds, slot);
        } else {
            const int k = item - n64 - i16 - i8;
            do_group<R, 1, false>(a, n64 + n16 + n8 + kWave * k, min(kWave, n1 - kWave * k), lds, slot);
        }
    }
}

template <int R, int P, bool WIDE>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2))) void k_plain(Args a, int first, int count)
{
    constexpr int G = kWave / P;
    extern __shared__ __align__(16) uint8_t lds[];
    uint32_t* slot = a.scratch + (int64_t)blockIdx.x * a.slot_words;
    first = max(first, 0);
    count = min(count, (int)a.n_pairs - first);
    const int items = (count + G - 1) / G;
    for (int k = blockIdx.x; k < items; k += gridDim.x)
        do_group<R, P, WIDE>(a, first + G * k, min(G, count - G * k), lds, slot);
}

// ASCII -> packed.  Thread t writes the 32 residues of high word t: positions
// [32 t - kGuardRes, 32 t + 32 - kGuardRes).
__global__ void k_pack(const uint8_t* __restrict__ ascii, int64_t n, uint32_t* __restrict__ blk,
                       int64_t n_hib_words, int32_t* err)
{
    // the letter -> code table in LDS: each residue is one LDS byte read
    // instead of a divergent load from constant memory
    __shared__ uint8_t tab[256];
    for (int i = threadIdx.x; i < 256; i += blockDim.x) tab[i] = c_tables.ascii[i];
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_hib_words) return;
    const int64_t p0 = 32 * t - kGuardRes;
    uint32_t nib[4] = {0, 0, 0, 0}, hib = 0;
    bool bad = false;
    auto put = [&](int k, uint32_t letter) {
        uint32_t c = tab[letter];
        if (c == 0xFFu) {
            c = kPadCode;
            bad = true;
        }
        nib[k >> 3] |= (c & 15u) << (4 * (k & 7));
        hib |= (c >> 4) << k;
    };
    if (p0 >= 0 && p0 + 32 <= n && ((reinterpret_cast<uintptr_t>(ascii) & 15u) == 0)) {
        // interior word: two 16-byte loads instead of 32 byte loads
        const uint4* src = reinterpret_cast<const uint4*>(ascii + p0);
        const uint4 v0 = src[0], v1 = src[1];
        const uint32_t w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
        for (int k = 0; k < 32; ++k) put(k, (w[k >> 2] >> (8 * (k & 3))) & 0xFFu);
    } else {
        for (int k = 0; k < 32; ++k) {
            const int64_t p = p0 + k;
            if (p >= 0 && p < n) {
                put(k, ascii[p]);
            } else {
                nib[k >> 3] |= (kPadCode & 15u) << (4 * (k & 7));
                hib |= (kPadCode >> 4) << k;
            }
        }
    }
    // nibble plane words 4t .. 4t+3, high plane word t (after n_hib_words * 4 nibble words)
    *reinterpret_cast<uint4*>(blk + 4 * t) = make_uint4(nib[0], nib[1], nib[2], nib[3]);
    blk[4 * n_hib_words + t] = hib;
    if (bad) atomicOr((unsigned*)err, (unsigned)kErrCode);
}

// ------------------------------------------------------------------ counting sort into cells
// Start-pass cell of a pair whose forward pass is done: by the reversed
// prefixes q[0..q_end], r[0..r_end]; -1 when there is nothing to do (score 0,
// or a pair the forward pass rejected).
__device__ __forceinline__ int classify_start(const Args& a, int64_t k)
{
    const sw_result r = a.out[k];
    if (r.score <= 0 || r.q_end < 0 || r.r_end < 0) return -1;
    return cell_of(a, (int64_t)r.q_end + 1, (int64_t)r.r_end + 1);
}

// Cell of pair k for its forward pass; -1 for pairs that need no work and -2
// for invalid pairs (the result of both is written here).
__device__ __forceinline__ int classify(const Args& a, int64_t k)
{
    const int64_t qi = a.pairs[2 * k], ri = a.pairs[2 * k + 1];
    sw_result bad;
    bad.score = bad.q_start = bad.q_end = bad.r_start = bad.r_end = -1;
    if (qi < 0 || qi >= a.n_q || ri < 0 || ri >= a.n_r) {
        a.out[k] = bad;
        return -2;
    }
    const int64_t q0 = a.q_offsets[qi], q1 = a.q_offsets[qi + 1], r0 = a.r_offsets[ri], r1 = a.r_offsets[ri + 1];
    if (q0 < 0 || r0 < 0 || q1 < q0 || r1 < r0 || q1 > a.qhdr->n_residues || r1 > a.rhdr->n_residues ||
        q1 - q0 > SW_MAX_SEQ_LEN || r1 - r0 > SW_MAX_SEQ_LEN) {
        a.out[k] = bad;
        return -2;
    }
    const int64_t m = q1 - q0, n = r1 - r0;
    if (m == 0 || n == 0) {
        sw_result z;
        z.score = 0;
        z.q_start = z.q_end = z.r_start = z.r_end = -1;
        a.out[k] = z;
        return -1;
    }
    return cell_of(a, m, n);
}

__global__ void k_fill(int32_t* p, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_zero_cells(Args a)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kNumCells * kCellShards; i += gridDim.x * blockDim.x)
        a.cell_count[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.counters[kCntHead] = 0;
}

// Classify each pair into its cell and reserve its place.  A block takes a
// tile of kPrepTile pairs: their counts per cell in LDS (an LDS atomic gives
// each pair its rank among the tile's pairs of its cell), then one global
// atomic per cell the tile holds reserves the tile's range on the cell's
// shard (the tile index mod kCellShards).  The global atomics, about 7 G/s
// one per pair, were the cost of this kernel.
constexpr int kPrepThreads = 1024;
constexpr int kPrepPer = 8;  // pairs per thread
constexpr int kPrepTile = kPrepThreads * kPrepPer;
__device__ __forceinline__ int pair_shard(int64_t k) { return (int)((k / kPrepTile) % kCellShards); }

__global__ __launch_bounds__(kPrepThreads) void k_prepare(Args a)
{
    __shared__ int hist[kNumCells];  // the tile's count of each cell, then its first rank on the shard
    for (int i = threadIdx.x; i < kNumCells; i += kPrepThreads) hist[i] = 0;
    __syncthreads();
    const int64_t k0 = (int64_t)blockIdx.x * kPrepTile + threadIdx.x;
    int cells[kPrepPer], local[kPrepPer];
    bool bad = false;
#pragma unroll
    for (int i = 0; i < kPrepPer; ++i) {
        const int64_t k = k0 + (int64_t)i * kPrepThreads;
        int cell = -1;
        if (k < a.n_pairs) {
            cell = a.phase == 2 ? classify_start(a, k) : classify(a, k);
            a.pair_cell[k] = cell;
            bad = bad || cell == -2;
        }
        cells[i] = cell;
        local[i] = cell >= 0 ? atomicAdd(&hist[cell], 1) : 0;
    }
    if (bad) atomicOr((unsigned*)a.err, (unsigned)kErrRange);
    __syncthreads();
    const int shard = (int)(blockIdx.x % kCellShards);
    for (int c = threadIdx.x; c < kNumCells; c += kPrepThreads) {
        const int cnt = hist[c];
        if (cnt > 0) hist[c] = atomicAdd(&a.cell_count[c * kCellShards + shard], cnt);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kPrepPer; ++i) {
        const int64_t k = k0 + (int64_t)i * kPrepThreads;
        if (cells[i] >= 0) a.pair_rank[k] = hist[cells[i]] + local[i];
    }
}

// Exclusive scan of the cell counts in rank order (a cell's shards in shard
// order): the counts become first positions, rank_start gets the first
// position of each rank, counters the number of pairs of each kind.  Two
// launches of kScanTiles blocks: each block sums its tile of kScanRanks
// ranks (all pairs, and those of 64-, 16- and 8-lane items), then each block
// scans its tile again from the sum of the tiles before it.
constexpr int kScanThreads = 256;
constexpr int kScanPer = kScanRanks / kScanThreads;  // ranks per thread
static_assert(kScanRanks % kScanThreads == 0, "whole ranks per thread");
static_assert(kCellShards == 16, "a cell's shards are read as four int4");

// this thread's ranks: their cells and counts (all shards)
__device__ __forceinline__ void scan_load(const Args& a, int tile, int (&cells)[kScanPer], int (&cnt)[kScanPer])
{
    const int r0 = tile * kScanRanks + threadIdx.x * kScanPer;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) cells[i] = r0 + i < kNumCells ? a.rank_cell[r0 + i] : 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        const int4* q = reinterpret_cast<const int4*>(a.cell_count + cells[i] * kCellShards);
        int c = 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int4 x = q[v];
            c += x.x + x.y + x.z + x.w;
        }
        cnt[i] = r0 + i < kNumCells ? c : 0;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(Args a)
{
    __shared__ int part[kScanThreads / kWave][4];
    int cells[kScanPer], cnt[kScanPer];
    scan_load(a, blockIdx.x, cells, cnt);
    int v[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        v[0] += cnt[i];
        const int kind = cell_kind(cells[i], a);
        v[1] += kind == 64 ? cnt[i] : 0;
        v[2] += kind == 16 ? cnt[i] : 0;
        v[3] += kind == 8 ? cnt[i] : 0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) v[k] += __shfl_xor(v[k], o, kWave);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) part[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 4) {
        int t = 0;
        for (int j = 0; j < kScanThreads / kWave; ++j) t += part[j][threadIdx.x];
        a.counters[kCntTiles + 4 * blockIdx.x + threadIdx.x] = t;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(Args a)
{
    __shared__ int wsum[kScanThreads / kWave];
    __shared__ int tile_base;
    const int tile = blockIdx.x;
    if (threadIdx.x == 0) {
        int b = 0;
        for (int j = 0; j < tile; ++j) b += a.counters[kCntTiles + 4 * j];
        tile_base = b;
    }
    int cells[kScanPer], cnt[kScanPer];
    scan_load(a, tile, cells, cnt);
    int mine = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) mine += cnt[i];
    // inclusive scan over the wave, then over the block's waves
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int inc = mine;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(inc, o, kWave);
        inc += lane >= o ? y : 0;
    }
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    int run = tile_base + inc - mine;
    for (int j = 0; j < w; ++j) run += wsum[j];
    const int r0 = tile * kScanRanks + threadIdx.x * kScanPer;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        if (r0 + i >= kNumCells) break;
        a.rank_start[r0 + i] = run;
        int4* q = reinterpret_cast<int4*>(a.cell_count + cells[i] * kCellShards);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int4 x = q[v];
            int4 y;
            y.x = run;
            y.y = run + x.x;
            y.z = y.y + x.y;
            y.w = y.z + x.z;
            run = y.w + x.w;
            q[v] = y;
        }
    }
    if (tile == kScanTiles - 1 && threadIdx.x == 0) {
        int t[4] = {0, 0, 0, 0};
        for (int j = 0; j < kScanTiles; ++j)
            for (int k = 0; k < 4; ++k) t[k] += a.counters[kCntTiles + 4 * j + k];
        a.rank_start[kNumCells] = t[0];
        a.counters[kCntP64] = t[1];
        a.counters[kCntP16] = t[2];
        a.counters[kCntP8] = t[3];
        a.counters[kCntP1] = t[0] - t[1] - t[2] - t[3];
        a.counters[kCntHead] = 0;  // the work queue of the launch that follows
    }
}

// Each pair to the place its classify reserved: the first position of its
// cell and shard (from the scan) plus its rank there.
__global__ void k_scatter(Args a)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.n_pairs;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int cell = a.pair_cell[k];
        if (cell >= 0) a.perm[a.cell_count[cell * kCellShards + pair_shard(k)] + a.pair_rank[k]] = (int32_t)k;
    }
}

// ------------------------------------------------------------------ launchers
size_t lds_bytes(int R) { return (size_t)kNumCodes * kWave * prof_bytes(R) + kXbufBytes; }

int64_t slot_words_for(int64_t max_len)
{
    const int64_t n = std::min<int64_t>(std::max<int64_t>(max_len, 0), SW_MAX_SEQ_LEN);
    const int64_t wide = n > kMaxP16Len ? 3 * wide_buf_words((int)n) : 0;
    return std::max(slot_words(), (wide + 63) & ~(int64_t)63);
}

int64_t slot_words()
{
    // [chunk][group][8 cells]: 64 groups of one lane over at most 128 chunks
    // (narrow, a ring of four buffers and the kept rows), 8 or 4 groups over
    // 512 chunks (8 or 16 lanes, narrow, three buffers), 1 group over 8192
    // chunks (64 lanes, wide, two words per cell; three buffers of the scan
    // fit up to ~54k columns)
    const int64_t p1 = (kKeptBuf + 1) * boundary_buf_words(1);
    const int64_t p8 = 3 * boundary_buf_words(8);
    const int64_t p16 = 3 * boundary_buf_words(16);
    const int64_t p64 = kWideBufWords;  // whole wave, longest pairs: one buffer, in place
    return std::max(std::max(p1, p8), std::max(p16, p64));
}

// ------------------------------------------------------------------ per-device arrays
// Tables every call reads (filled by the host at set-up) and the error word.
static __device__ __align__(256) int32_t g_rank_cell[2][kNumCells];
static __device__ __align__(256) int32_t g_err_word[64];
// Workspace of sw_align_sets_static (sort tables, pair arrays and boundary-row
// slots, carved as a caller's buffer would be), for callers that cannot
// allocate device memory.  Every device the library is loaded on holds its
// own copy until the process ends; every call on a device shares it.
static __device__ __align__(256) uint8_t scratch[kStaticWsBytes];

hipError_t device_statics(DeviceStatics* s)
{
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_rank_cell));
    if (e != hipSuccess) return e;
    s->rank_cell_persistent = static_cast<int32_t*>(p);
    s->rank_cell_plain = static_cast<int32_t*>(p) + kNumCells;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_err_word));
    if (e != hipSuccess) return e;
    s->err = static_cast<int32_t*>(p);
    // host code uses this address, never the array's own name (a host-side
    // stand-in that is not a device address)
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    s->static_ws = p;
    return hipSuccess;
}

__global__ void k_pack_header(PackedHeader* h, int64_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        h->magic = kPackMagic;
        h->version = 2;  // planar: nibble plane, then high plane
        h->n_residues = n;
        h->n_blocks = (kGuardRes + n + kTailRes + 255) / 256 + 1;
        h->total_bytes = kHeaderBytes + h->n_blocks * 160;
    }
}

hipError_t launch_pack(const char* ascii, int64_t n, void* packed, int32_t* err, hipStream_t stream)
{
    PackedHeader* h = reinterpret_cast<PackedHeader*>(packed);
    uint32_t* blk = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(packed) + kHeaderBytes);
    const int64_t n_hib_words = packed_blocks(n) * 8;
    const int threads = 256;
    const int64_t blocks = (n_hib_words + threads - 1) / threads;
    hipLaunchKernelGGL(k_pack_header, dim3(1), dim3(64), 0, stream, h, n);
    hipLaunchKernelGGL(k_pack, dim3((unsigned)blocks), dim3(threads), 0, stream, (const uint8_t*)ascii, n, blk,
                       n_hib_words, err);
    return hipGetLastError();
}

hipError_t launch_prepare(const Args& a, hipStream_t stream)
{
    const int64_t blocks = std::min<int64_t>((a.n_pairs + 255) / 256, 4096);
    const int64_t tiles = (a.n_pairs + kPrepTile - 1) / kPrepTile;
    hipLaunchKernelGGL(k_zero_cells, dim3(64), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_prepare, dim3((unsigned)std::max<int64_t>(tiles, 1)), dim3(kPrepThreads), 0, stream, a);
    hipLaunchKernelGGL(k_scan_tiles, dim3(kScanTiles), dim3(kScanThreads), 0, stream, a);
    hipLaunchKernelGGL(k_scan_apply, dim3(kScanTiles), dim3(kScanThreads), 0, stream, a);
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, stream, a);
    return hipGetLastError();
}

template <int R>
static hipError_t launch_persistent_r(const Args& a, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(k_persistent<R>, dim3(grid), dim3(kWave), lds_bytes(R), stream, a);
    return hipGetLastError();
}

hipError_t launch_persistent(const Args& a, int grid, hipStream_t stream)
{
    switch (a.rows_per_lane) {
    case 8: return launch_persistent_r<8>(a, grid, stream);
    case 16: return launch_persistent_r<16>(a, grid, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int R>
static hipError_t launch_plain_r(const Args& a, int kind, int first, int count, int grid, hipStream_t stream)
{
    const size_t lds = lds_bytes(R);
    if (kind == 64)
        hipLaunchKernelGGL((k_plain<R, 64, true>), dim3(grid), dim3(kWave), lds, stream, a, first, count);
    else if (kind == 16)
        hipLaunchKernelGGL((k_plain<R, 16, false>), dim3(grid), dim3(kWave), lds, stream, a, first, count);
    else if (kind == 8)
        hipLaunchKernelGGL((k_plain<R, 8, false>), dim3(grid), dim3(kWave), lds, stream, a, first, count);
    else
        hipLaunchKernelGGL((k_plain<R, 1, false>), dim3(grid), dim3(kWave), lds, stream, a, first, count);
    return hipGetLastError();
}

hipError_t launch_plain(const Args& a, int kind, int first, int count, int grid, hipStream_t stream)
{
    switch (a.rows_per_lane) {
    case 8: return launch_plain_r<8>(a, kind, first, count, grid, stream);
    case 16: return launch_plain_r<16>(a, kind, first, count, grid, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int R>
static hipError_t set_attrs_r()
{
    const int bytes = (int)lds_bytes(R);
    const hipFuncAttribute at = hipFuncAttributeMaxDynamicSharedMemorySize;
    hipError_t e = hipFuncSetAttribute((const void*)k_persistent<R>, at, bytes);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_plain<R, 1, false>, at, bytes);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_plain<R, 16, false>, at, bytes);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_plain<R, 8, false>, at, bytes);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_plain<R, 64, true>, at, bytes);
    return e;
}

hipError_t set_kernel_attributes()
{
    hipError_t e = set_attrs_r<16>();
    return e == hipSuccess ? set_attrs_r<8>() : e;
}

}  // namespace swk
