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
// Cell update used everywhere (8-9 VALU instructions per cell):
//   d  = H[i-1][j-1] + s(q_i, r_j)           one SDWA add (profile byte, sign-extended)
//   H  = max3(d, E[i][j], F[i][j])           E, F >= 0, so H >= 0 is the local floor
//   hg = sat(H - go)                         v_sub_u32 clamp
//   E[i][j+1] = max(E[i][j] - ge, hg)        hg >= 0 keeps E >= 0
//   F[i+1][j] = max(F[i][j] - ge, hg)
//   K[r] = max(K[r], H << TB | tag(j))       per-row best with the earliest column
// Keeping E and F saturated at 0 leaves H exactly as in the textbook
// recurrence: by induction E_sat = max(E, 0), and H only uses max(0, E).
//
// Kernel body: one pair per lane.  The lane keeps R query rows in registers
// and sweeps the reference; horizontal strips of R rows hand their bottom row
// to the next strip through a per-block scratch slot; the substitution scores
// come from a per-lane query profile in LDS.  Two variants: "narrow" for
// pairs whose scores fit 16 bits (one dword per boundary cell, 16-bit column
// tags) and "wide" for any pair up to the length limit (two dwords per
// boundary cell, 12-bit column tags folded every 4096 columns).

#include <algorithm>

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

struct CodeTables {
    uint32_t tab[kNumCodes][8];  // row c: bytes s(c, x) for x = 0..31 (pad and unused: -128)
    uint8_t ascii[256];          // ASCII -> code, 0xFF if not a symbol
};

static constexpr CodeTables make_tables()
{
    CodeTables t{};
    for (int a = 0; a < kNumCodes; ++a)
        for (int w = 0; w < 8; ++w) {
            uint32_t word = 0;
            for (int k = 0; k < 4; ++k) {
                int b = 4 * w + k;
                int v = -128;
                if (a < kNumSym && b < kNumSym)
                    v = kBlosum62Ncbi[ncbi_index(kCodeOrder[a])][ncbi_index(kCodeOrder[b])];
                word |= (uint32_t)(uint8_t)(int8_t)v << (8 * k);
            }
            t.tab[a][w] = word;
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
// Word of the nibble / high plane holding residue p (p may be as low as
// -kGuardRes).  Planes are interleaved in 256-residue blocks of 40 words.
__device__ __forceinline__ int64_t nib_word(int64_t p)
{
    int64_t q = p + kGuardRes;
    return (q >> 8) * 40 + ((q >> 3) & 31);
}
__device__ __forceinline__ int64_t hib_word(int64_t p)
{
    int64_t q = p + kGuardRes;
    return (q >> 8) * 40 + 32 + ((q >> 5) & 7);
}

// A sequence view: residues B + x for x >= -256 addressed with 32-bit offsets
// from the block before the one holding B.
struct SeqView {
    const uint32_t* ptr;
    int off;
};

__device__ __forceinline__ SeqView seq_view(const uint32_t* __restrict__ blk, int64_t B)
{
    const int64_t q = B + kGuardRes;
    SeqView v;
    v.ptr = blk + ((q >> 8) - 1) * 40;
    v.off = (int)(q & 255) + 256;
    return v;
}

__device__ __forceinline__ int view_nib(int q) { return (q >> 8) * 40 + ((q >> 3) & 31); }
__device__ __forceinline__ int view_hib(int q) { return (q >> 8) * 40 + 32 + ((q >> 5) & 7); }

// Codes of the 8 residues B+x .. B+x+7: nibble k of nw, bit k of hw.
__device__ __forceinline__ void window8(const SeqView& v, int x, uint32_t& nw, uint32_t& hw)
{
    const int q = v.off + x;
    const uint32_t a0 = v.ptr[view_nib(q)], a1 = v.ptr[view_nib(q + 8)];
    nw = __builtin_amdgcn_alignbit(a1, a0, (uint32_t)(q & 7) * 4u);
    const uint32_t b0 = v.ptr[view_hib(q)], b1 = v.ptr[view_hib(q + 32)];
    hw = __builtin_amdgcn_alignbit(b1, b0, (uint32_t)(q & 31));
}

// Code of the single residue B + x.
__device__ __forceinline__ uint32_t code_at(const SeqView& v, int x)
{
    const int q = v.off + x;
    return ((v.ptr[view_nib(q)] >> ((q & 7) * 4)) & 15u) | (((v.ptr[view_hib(q)] >> (q & 31)) & 1u) << 4);
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
// Layout [code][lane][R bytes]: lane l's scores for its R rows against a
// reference residue `code` are 8 or 16 contiguous bytes; a wave's reads of
// one row of the layout are contiguous in lane order, so the 8- or 16-byte
// reads are conflict-free whatever codes the lanes hold.

// One profile entry (R bytes) as 16-byte stores, or one 8-byte store for R = 8.
template <int R>
__device__ __forceinline__ void store_entry(uint8_t* dst, const uint32_t (&v)[R / 4])
{
    if constexpr (R == 8) {
        *reinterpret_cast<uint2*>(dst) = make_uint2(v[0], v[1]);
    } else {
        uint4* d4 = reinterpret_cast<uint4*>(dst);
#pragma unroll
        for (int w = 0; w < R / 16; ++w) d4[w] = make_uint4(v[4 * w], v[4 * w + 1], v[4 * w + 2], v[4 * w + 3]);
    }
}

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
    uint8_t* base = prof + lane * R;
#pragma unroll 1
    for (int c = 0; c < kNumSym; ++c) {
        const uint32_t* t = c_tables.tab[c];
        const uint32_t t0 = t[0], t1 = t[1], t2 = t[2], t3 = t[3], t4 = t[4], t5 = t[5];
        uint32_t v[R / 4];
#pragma unroll
        for (int w = 0; w < R / 4; ++w)
            v[w] = __builtin_amdgcn_perm(t1, t0, sel[w][0]) | __builtin_amdgcn_perm(t3, t2, sel[w][1]) |
                   __builtin_amdgcn_perm(t5, t4, sel[w][2]);
        store_entry<R>(base + c * (kWave * R), v);
    }
    uint32_t pad[R / 4];
#pragma unroll
    for (int w = 0; w < R / 4; ++w) pad[w] = 0x80808080u;
    store_entry<R>(base + kPadCode * (kWave * R), pad);
}

template <int R>
__device__ __forceinline__ void load_profile(const uint8_t* prof_lane, uint32_t code, uint32_t (&w)[R / 4])
{
    if constexpr (R == 8) {
        const uint2 v = *reinterpret_cast<const uint2*>(prof_lane + code * (uint32_t)(kWave * R));
        w[0] = v.x;
        w[1] = v.y;
        return;
    }
    const uint4* p = reinterpret_cast<const uint4*>(prof_lane + code * (uint32_t)(kWave * R));
#pragma unroll
    for (int k = 0; k < R / 16; ++k) {
        const uint4 v = p[k];
        w[4 * k] = v.x;
        w[4 * k + 1] = v.y;
        w[4 * k + 2] = v.z;
        w[4 * k + 3] = v.w;
    }
}

// ------------------------------------------------------------------ the cell update
// h + sign_extend(byte SEL of w), one v_add_u32 with an SDWA byte operand.
template <int SEL>
__device__ __forceinline__ int add_sbyte(int h, uint32_t w)
{
    return h + (int)(int8_t)(uint8_t)(w >> (8 * SEL));
}

// Hides what the compiler knows about the value's range (no instruction).
// E and F are never negative; once the compiler proves that, it splits
// max(max(d, E), F) into a signed and an unsigned max instead of one
// v_max3_i32.
__device__ __forceinline__ void opaque(int& v) { asm("" : "+v"(v)); }

template <int R, int I>
struct RowUnroll {
    template <int TB>
    static __device__ __forceinline__ void run(int (&H)[R], int (&E)[R], uint32_t (&K)[R],
                                               const uint32_t (&w)[R / 4], int& d, int& F,
                                               uint32_t tag, uint32_t go, int ge)
    {
        int dn = 0;
        if constexpr (I + 1 < R) dn = add_sbyte<(I + 1) & 3>(H[I], w[(I + 1) >> 2]);
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

// One column of a lane's R rows.  hdiag = H[row0-1][j-1]; F enters as
// F[row0][j] and leaves as F[row0+R][j].
template <int R, int TB>
__device__ __forceinline__ void column_step(int (&H)[R], int (&E)[R], uint32_t (&K)[R],
                                            const uint32_t (&w)[R / 4], int hdiag, int& F,
                                            uint32_t tag, uint32_t go, int ge)
{
    int d = add_sbyte<0>(hdiag, w[0]);
    RowUnroll<R, 0>::template run<TB>(H, E, K, w, d, F, tag, go, ge);
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

template <int R, int P, bool REV, bool WIDE>
__device__ Best group_sweep(const Args& a, uint8_t* prof, uint4* xbuf, uint32_t* __restrict__ slot,
                            int64_t Q0, int M, int64_t R0, int N, int target)
{
    constexpr int TB = WIDE ? 12 : 16;  // tag bits of the per-row trackers
    constexpr int SW = WIDE ? 4 : 2;    // uint4 per boundary chunk of 8 columns
    constexpr int G = kWave / P;        // groups per wave
    const int lane = threadIdx.x & (kWave - 1);
    const int u = lane % P, g = lane / P;
    const uint8_t* prof_lane = prof + lane * R;
    const uint32_t go = (uint32_t)a.go;
    const int ge = a.ge;
    Best b{0, -1, -1};  // this lane's rows only
    const int my_ss = (M > 0 && N > 0) ? (M + P * R - 1) / (P * R) : 0;
    const int my_chunks = (N + 7) / 8;
    const int wss = uni(wave_max(my_ss));
    const int wc = uni(wave_max(my_ss > 0 ? my_chunks : 0));
    bool done = my_ss == 0 || (REV && target <= 0);
    const SeqView qv = seq_view(a.qblk, Q0);
    const SeqView rv = seq_view(a.rblk, R0);
    uint4* slot4 = reinterpret_cast<uint4*>(slot) + SW * g;
    uint4* x_mine = xbuf + SW * lane;
    const uint4* x_up = xbuf + SW * (lane > 0 ? lane - 1 : 0);

#pragma unroll 1
    for (int ss = 0; ss < wss; ++ss) {
        if (__ballot(!done && ss < my_ss) == 0) break;
        const bool gact = !done && ss < my_ss;
        const int row0 = ss * P * R + u * R;
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
        const bool read_top = ss > 0;            // uniform
        const bool write_next = ss + 1 < my_ss;  // uniform within the group

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
        uint4 tc_n[SW];
        uint32_t nw_n, hw_n;
        auto fetch = [&](int cn) {
            if (u == 0) {
                const int cc = min(max(cn, 0), max(my_chunks - 1, 0));
#pragma unroll
                for (int w = 0; w < SW; ++w)
                    tc_n[w] = read_top ? slot4[cc * G * SW + w] : make_uint4(0, 0, 0, 0);
            }
            window8(rv, chunk_x(cn), nw_n, hw_n);
        };
        fetch(-u);
#pragma unroll 1
        for (int t = 0; t < T; ++t) {
            const int c = t - u;
            const bool act = gact && c >= 0 && c < my_chunks;
            uint4 tc[SW];
#pragma unroll
            for (int w = 0; w < SW; ++w) tc[w] = u == 0 ? tc_n[w] : x_up[w];
            uint32_t nw = nw_n, hw = hw_n;
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
                uint32_t w[R / 4];
                load_profile<R>(prof_lane, code_of(0), w);
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    uint32_t wn[R / 4];
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
                        for (int i = 0; i < R / 4; ++i) w[i] = wn[i];
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
                    slot4[c * G * SW + w] = make_uint4(bot[4 * w], bot[4 * w + 1], bot[4 * w + 2], bot[4 * w + 3]);
            }
            if constexpr (WIDE) {
                if ((t & 511) == 511) fold(8 * t + 7 - 4095);
            }
        }
        block_fence();
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
    return group_best<P>(b);
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

// One work item: up to 64/P pairs, P lanes each.
template <int R, int P, bool WIDE>
__device__ void do_group(const Args& a, int first, int count, uint8_t* lds, uint32_t* slot)
{
    constexpr int G = kWave / P;
    constexpr int SW = WIDE ? 4 : 2;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / P, u = lane % P;
    int pid = -1, m = 0, n = 0;
    int64_t qoff = 0, roff = 0;
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
        // the slot must hold one boundary cell per column for every group
        const int64_t need = (int64_t)((n + 7) / 8) * G * SW * 4;
        if (need > a.slot_words) {
            if (u == 0) {
                atomicOr((unsigned*)a.err, (unsigned)kErrInternal);
                sw_result bad;
                bad.score = bad.q_start = bad.q_end = bad.r_start = bad.r_end = -1;
                a.out[pid] = bad;
            }
            pid = -1;
            m = n = 0;
        }
    }
    uint8_t* prof = lds;
    uint4* xbuf = reinterpret_cast<uint4*>(lds + kNumCodes * kWave * R);
    const Best f = group_sweep<R, P, false, WIDE>(a, prof, xbuf, slot, qoff, m, roff, n, 0);
    const bool has = f.s > 0;
    const Best r = group_sweep<R, P, true, WIDE>(a, prof, xbuf, slot, qoff + (has ? f.i : 0), has ? f.i + 1 : 0,
                                                 roff + (has ? f.j : 0), has ? f.j + 1 : 0, f.s);
    if (pid >= 0 && u == 0) {
        if (has && r.s != f.s) atomicOr((unsigned*)a.err, (unsigned)kErrInternal);
        write_result(a.out, pid, f.s, f.i - r.i, f.i, f.j - r.j, f.j);
    }
}

// ------------------------------------------------------------------ kernels
// Work items, in queue order: single pairs over 64 lanes (longest first),
// groups of 4 pairs over 16 lanes each, groups of 64 pairs one per lane.
template <int R>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2))) void k_persistent(Args a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    uint32_t* slot = a.scratch + (int64_t)blockIdx.x * a.slot_words;
    // the counters come from the scan; clamp them so that a bookkeeping error
    // can never index past the permutation
    const int n64 = min(max(a.counters[kCntP64], 0), (int)a.n_pairs);
    const int n16 = min(max(a.counters[kCntP16], 0), (int)a.n_pairs - n64);
    const int n1 = min(max(a.counters[kCntP1], 0), (int)a.n_pairs - n64 - n16);
    const int i16 = (n16 + 3) / 4, i1 = (n1 + kWave - 1) / kWave;
    const int total = n64 + i16 + i1;
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
        } else {
            const int k = item - n64 - i16;
            do_group<R, 1, false>(a, n64 + n16 + kWave * k, min(kWave, n1 - kWave * k), lds, slot);
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
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_hib_words) return;
    const int64_t p0 = 32 * t - kGuardRes;
    uint32_t nib[4] = {0, 0, 0, 0}, hib = 0;
    bool bad = false;
    for (int k = 0; k < 32; ++k) {
        const int64_t p = p0 + k;
        uint32_t c = kPadCode;
        if (p >= 0 && p < n) {
            c = c_tables.ascii[ascii[p]];
            if (c == 0xFFu) {
                c = kPadCode;
                bad = true;
            }
        }
        nib[k >> 3] |= (c & 15u) << (4 * (k & 7));
        hib |= (c >> 4) << k;
    }
    const int64_t blkidx = t >> 3, sub = t & 7;  // 8 high words (256 residues) per block
    uint32_t* b = blk + blkidx * 40;
    for (int k = 0; k < 4; ++k) b[4 * sub + k] = nib[k];
    b[32 + sub] = hib;
    if (bad) atomicOr((unsigned*)err, (unsigned)kErrCode);
}

// ------------------------------------------------------------------ work cells
__device__ __forceinline__ int ceil_log2(int64_t x)
{
    int b = 0;
    while (((int64_t)1 << b) < x) ++b;
    return b;
}

// Lanes per pair of a work cell: 1 for the short-pair cells, 16 for long
// pairs up to kMaxP16Len residues, 64 beyond.
__device__ __forceinline__ int cell_kind(int cell)
{
    if (cell < kInterCells) return 1;
    const int bucket = (cell - kInterCells) / kWideCostBins;
    return (1 << bucket) <= kMaxP16Len ? 16 : 64;
}

// Cell of a pair: lane-per-pair pairs by (strips, chunks), long pairs by
// (length bucket, 16*log2(m*n)).  Returns -1 for pairs that need no work and
// -2 for invalid pairs (their result is written here).
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
    const int64_t mx = m > n ? m : n;
    if (mx <= a.inter_max_len) {
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

__global__ void k_fill(int32_t* p, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_zero_cells(Args a)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kNumCells; i += gridDim.x * blockDim.x)
        a.cell_count[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.counters[kCntHead] = 0;
}

__global__ void k_prepare(Args a)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.n_pairs;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int cell = classify(a, k);
        a.pair_cell[k] = cell;
        if (cell >= 0) atomicAdd(&a.cell_count[cell], 1);
        else if (cell == -2) atomicOr((unsigned*)a.err, (unsigned)kErrRange);
    }
}

// Single block: exclusive scan of the cell counts in rank order; the counts
// become scatter cursors; counters get the number of long and short pairs.
__global__ __launch_bounds__(1024) void k_scan(Args a)
{
    __shared__ int part[1024];
    __shared__ int n64s[1024];
    __shared__ int n16s[1024];
    const int t = threadIdx.x;
    constexpr int per = (kNumCells + 1023) / 1024;
    const int lo = t * per, hi = min(kNumCells, lo + per);
    int sum = 0, c64 = 0, c16 = 0;
    for (int rk = lo; rk < hi; ++rk) {
        const int cell = a.rank_cell[rk];
        const int c = a.cell_count[cell];
        sum += c;
        const int kind = cell_kind(cell);
        if (kind == 64) c64 += c;
        else if (kind == 16) c16 += c;
    }
    part[t] = sum;
    n64s[t] = c64;
    n16s[t] = c16;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int v = t >= o ? part[t - o] : 0;
        const int w = t >= o ? n64s[t - o] : 0;
        const int x = t >= o ? n16s[t - o] : 0;
        __syncthreads();
        part[t] += v;
        n64s[t] += w;
        n16s[t] += x;
        __syncthreads();
    }
    int run = part[t] - sum;  // exclusive prefix
    for (int rk = lo; rk < hi; ++rk) {
        const int cell = a.rank_cell[rk];
        const int c = a.cell_count[cell];
        a.rank_start[rk] = run;
        a.cell_count[cell] = run;
        run += c;
    }
    if (t == 1023) {
        a.rank_start[kNumCells] = part[1023];
        a.counters[kCntP64] = n64s[1023];
        a.counters[kCntP16] = n16s[1023];
        a.counters[kCntP1] = part[1023] - n64s[1023] - n16s[1023];
    }
}

__global__ void k_scatter(Args a)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.n_pairs;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int cell = a.pair_cell[k];
        if (cell >= 0) a.perm[atomicAdd(&a.cell_count[cell], 1)] = (int32_t)k;
    }
}

// ------------------------------------------------------------------ launchers
size_t lds_bytes(int R) { return (size_t)kNumCodes * kWave * R + kXbufBytes; }

int64_t slot_words()
{
    // [chunk][group][8 cells]: 64 groups of one lane over at most 128 chunks
    // (narrow), 4 groups over 512 chunks (16 lanes, narrow), 1 group over
    // 8192 chunks (64 lanes, wide, two words per cell)
    const int64_t p1 = (int64_t)kMaxInterChunks * 64 * 8;
    const int64_t p16 = (int64_t)(kMaxP16Len / 8) * 4 * 8;
    const int64_t p64 = (int64_t)((SW_MAX_SEQ_LEN + 7) / 8) * 1 * 16;
    return std::max(p1, std::max(p16, p64));
}

__global__ void k_pack_header(PackedHeader* h, int64_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        h->magic = kPackMagic;
        h->version = 1;
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
    hipLaunchKernelGGL(k_zero_cells, dim3(64), dim3(256), 0, stream, a);
    const int64_t blocks = std::min<int64_t>((a.n_pairs + 255) / 256, 4096);
    hipLaunchKernelGGL(k_prepare, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, stream, a);
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
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_plain<R, 64, true>, at, bytes);
    return e;
}

hipError_t set_kernel_attributes()
{
    hipError_t e = set_attrs_r<16>();
    return e == hipSuccess ? set_attrs_r<8>() : e;
}

}  // namespace swk
