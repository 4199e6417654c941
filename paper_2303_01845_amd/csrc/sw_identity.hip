// Identity and coverage of aligned pairs: the numbers the similarity-graph
// filter keeps an edge by.
//
// The paper forms the similarity graph from alignment metrics -- identity and
// coverage -- kept above thresholds (section "Protein similarity search
// pipeline"; thresholds 0.30 and 0.70 in the program parameters of section
// "Similarity search at scale").  Identity depends on which optimal alignment
// is taken; this pass takes, over the box the aligner reported
// (q[q_start..q_end] x r[r_start..r_end]), the global alignment that is best
// first by score, then by the number of identical pairs, then by the fewest
// columns, and reports its matches and columns.
//
// One wave per pair, pairs handed out by a counter.  The box is swept in
// strips of 64 R rows (R rows per lane): lane l owns rows base + R l ..
// + R - 1 and at step t computes column t - l of all of them, so the cells
// above its first row come from lane l-1's previous two steps by lane
// shuffles, and each further row reads the one above it in registers (R
// cells per step share the shuffles and the loop overhead).  R is 4 for
// every full 256-row strip and, for the box's last strip, the smallest of 1,
// 2 or 4 that covers its rows: a strip costs the wave about N steps of R
// cells per lane whatever its height.  The strip's bottom row (H and F) goes
// to the wave's scratch row in global memory for the next strip; lane 0 reads
// it 64 columns at a time, one chunk ahead, as it reads the reference codes.
//
// Each state holds one 64-bit key that orders alignments exactly as wanted:
//   key = score << 40 | matches << 20 | (2^20 - 1 - columns)
// Scores of kept cells are positive and below 2^20, matches and columns below
// 2^20, so the fields never borrow from one another and integer order of keys
// is the wanted lexicographic order; keys add along a path.  A cell whose
// best score is not positive is dropped (key -2^62): every proper prefix of
// an optimal alignment that starts at the reported start scores above zero
// (otherwise a later start would be optimal too, and the reported start is
// the latest one), so no dropped cell lies on an alignment that can win.
#include <algorithm>
#include <type_traits>

#include "identity_internal.h"

namespace swk {

namespace {

constexpr int64_t kNegKey = -(int64_t(1) << 62);
constexpr int kScoreShift = 40;
constexpr int kMatchShift = 20;
constexpr int64_t kFieldMask = (int64_t(1) << 20) - 1;
constexpr int64_t kOriginKey = kFieldMask;  // score 0, no matches, no columns

__device__ __forceinline__ uint32_t code_at(const uint32_t* __restrict__ nib, const uint32_t* __restrict__ hib,
                                            int64_t pos)
{
    const int64_t q = pos + kGuardRes;
    const uint32_t lo = (nib[q >> 3] >> (4 * (uint32_t)(q & 7))) & 15u;
    const uint32_t hi = (hib[q >> 5] >> (uint32_t)(q & 31)) & 1u;
    return lo | (hi << 4);
}

__device__ __forceinline__ int64_t cut(int64_t k) { return (k >> kScoreShift) > 0 ? k : kNegKey; }
__device__ __forceinline__ int64_t kmax(int64_t a, int64_t b) { return a > b ? a : b; }

__device__ __forceinline__ int64_t shfl_up64(int64_t v)
{
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)u, 1, 64);
    const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(u >> 32), 1, 64);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Value of lane `src` (wave-uniform) on every lane, without going through LDS.
__device__ __forceinline__ uint32_t readlane32(uint32_t v, int src)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, src);
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int src)
{
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = readlane32((uint32_t)u, src);
    const uint32_t hi = readlane32((uint32_t)(u >> 32), src);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Sweep rows row0 .. row1 - 1 of an M-row box in strips of 64 R rows (R rows
// per lane; the rows above row0 were swept before, their last row in the
// wave's scratch row) and return the key of the box's last cell on the lane
// that owns it (kNegKey on the others, and when row1 < M).
template <int R>
__device__ __forceinline__ int64_t sweep_box(const int8_t* sub, int64_t* Hrow, int64_t* Frow,
                                             const uint32_t* qnib, const uint32_t* qhib, const uint32_t* rnib,
                                             const uint32_t* rhib, int64_t GO, int64_t GE, int M, int N,
                                             int64_t Q0, int64_t R0, int lane, bool& bad_code, int row0, int row1)
{
    constexpr int kStrip = 64 * R;
    const int n_strips = (row1 - row0 + kStrip - 1) / kStrip;
    int64_t fin = kNegKey;
    for (int st = 0; st < n_strips; ++st) {
        // lane l owns rows i0 .. i0 + R - 1 of the strip
        const int base = row0 + st * kStrip;
        const int rows = min(kStrip, row1 - base);
        const int i0 = base + R * lane;
        const bool ok0 = R * lane < rows;
        const int8_t* subr[R];
        uint32_t qcr[R];
        int64_t E[R], Hleft[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            uint32_t qc = R * lane + r < rows ? code_at(qnib, qhib, Q0 + i0 + r) : 0u;
            if (qc >= (uint32_t)kNumSym) {
                bad_code = true;
                qc = 0;
            }
            qcr[r] = qc;
            subr[r] = sub + qc * kNumSym;
            E[r] = kNegKey;
            Hleft[r] = kNegKey;
        }
        int64_t diag_next = (lane == 0 && base == 0) ? kOriginKey : kNegKey;
        int64_t outH = kNegKey, outF = kNegKey;  // the lane's last row, handed to lane l+1
        uint32_t rc_prev = 0;
        // reference codes and the row above, 64 columns per chunk, one
        // chunk ahead (reads past the box stay inside the padded buffer
        // and the wave's scratch row; their values are never used)
        uint32_t cur = code_at(rnib, rhib, R0 + lane);
        uint32_t nxt = code_at(rnib, rhib, R0 + 64 + lane);
        const bool above = base > 0;
        int64_t curH = kNegKey, curF = kNegKey, nxtH = kNegKey, nxtF = kNegKey;
        if (above) {
            curH = Hrow[lane];
            curF = Frow[lane];
            nxtH = Hrow[min(64 + lane, kIdentMaxCols - 1)];
            nxtF = Frow[min(64 + lane, kIdentMaxCols - 1)];
        }
        const int lanes_used = (rows + R - 1) / R;
        const int steps = N + lanes_used - 1;
        for (int t = 0; t < steps; ++t) {
            if (t > 0 && (t & 63) == 0) {
                cur = nxt;
                nxt = code_at(rnib, rhib, R0 + t + 64 + lane);
                if (above) {
                    curH = nxtH;
                    curF = nxtF;
                    const int c = min(t + 64 + lane, kIdentMaxCols - 1);
                    nxtH = Hrow[c];
                    nxtF = Frow[c];
                }
            }
            // lane 0's inputs (the new column's code, the row above) are
            // read from one lane of the chunk; every other lane takes its
            // left neighbour's values of the previous step
            const int src = t & 63;
            const uint32_t rc_new = readlane32(cur, src);
            const uint32_t rc_up = (uint32_t)__shfl_up((int)rc_prev, 1, 64);
            const uint32_t rc = lane == 0 ? rc_new : rc_up;
            rc_prev = rc;
            int64_t upH = shfl_up64(outH);
            int64_t upF = shfl_up64(outF);
            const int64_t topH = readlane64(curH, src);
            const int64_t topF = readlane64(curF, src);
            if (lane == 0) {
                upH = (above && t < N) ? topH : kNegKey;
                upF = (above && t < N) ? topF : kNegKey;
            }
            const int64_t diag = diag_next;
            diag_next = upH;
            const int j = t - lane;
            if (ok0 && j >= 0 && j < N) {
                uint32_t rcc = rc;
                if (rcc >= (uint32_t)kNumSym) {
                    bad_code = true;
                    rcc = 0;
                }
                // row by row down the lane: the row above is the one just
                // computed, the above-left cell its value one column back
                int64_t dg = diag;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int64_t sc = (int64_t)subr[r][rcc];
                    const int64_t step = (sc << kScoreShift) + (qcr[r] == rcc ? (int64_t(1) << kMatchShift) : 0) - 1;
                    const int64_t d = cut(dg + step);
                    E[r] = cut(kmax(E[r] + GE, Hleft[r] + GO));
                    const int64_t F = cut(kmax(upF + GE, upH + GO));
                    const int64_t H = kmax(d, kmax(E[r], F));
                    dg = Hleft[r];
                    Hleft[r] = H;
                    upH = H;
                    upF = F;
                    if (j == N - 1 && i0 + r == M - 1) fin = H;
                }
                outH = upH;
                outF = upF;
                if (lane == 63 && base + kStrip < M) {  // a full strip with rows below it
                    Hrow[j] = upH;
                    Frow[j] = upF;
                }
            } else {
                outH = kNegKey;
                outF = kNegKey;
            }
        }
        // the strip's bottom row is in memory before the next strip reads it
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt and lgkmcnt untouched
    }
    return fin;
}

// ---------------------------------------------------------------- 32-bit keys
// Boxes of at most 511 x 511 residues (with gap penalties small enough, see
// box32_ok) run the same wavefront with one 32-bit key per state:
//   key = score << 18 | matches << 9 | pairs
// where pairs counts aligned pairs.  A global alignment of an M x N box has
// M + N - pairs columns, so most pairs is fewest columns and integer order of
// keys is again the wanted lexicographic order (score, matches, -columns);
// matches and pairs stay below 2^9, so the fields never borrow and keys add
// along a path, for scores of either sign.  No cell is dropped: the row above
// the box and the column left of it hold the exact keys of leading gaps
// (score -(go + k ge)), so every value is the key of a real path from the
// box's origin, and the states that cannot exist there (E left of the box, F
// above it) are a constant that loses every maximum.  Every value then lies
// within the bounds box32_ok checks.  A diagonal step adds one entry of a
// 24 x 24 table in LDS (score, match and pair together).
constexpr int kKey32ScoreShift = 18;
constexpr int kKey32MatchShift = 9;
constexpr int kKey32Field = 511;
constexpr int32_t kNegKey32 = -(1 << 30);

// The two exact key formats: 32-bit (score, matches, pairs) for small boxes,
// and the 64-bit (score, matches, 2^20 - 1 - columns) of the dropping sweep
// above, here with exact borders and nothing dropped, for the boxes whose
// values fit its score field (box64x_ok).
struct Key32 {
    typedef int32_t T;
    static constexpr T kNeg = kNegKey32;
    // a leading gap of k + 1 residues: its score, no pairs
    static __device__ __forceinline__ T gap(int64_t go, int64_t ge, int64_t k)
    {
        return -(T)((go + k * ge) << kKey32ScoreShift);
    }
    static __device__ __forceinline__ T step(int64_t g) { return -(T)(g << kKey32ScoreShift); }
    static __device__ __forceinline__ T up(T v) { return __shfl_up(v, 1, 64); }
    static __device__ __forceinline__ T mx(T a, T b) { return a > b ? a : b; }
    static __device__ __forceinline__ T lane_value(T v, int src) { return (T)readlane32((uint32_t)v, src); }
};

struct Key64 {
    typedef int64_t T;
    static constexpr T kNeg = kNegKey;
    // a leading gap of k + 1 residues: its score and k + 1 columns
    static __device__ __forceinline__ T gap(int64_t go, int64_t ge, int64_t k)
    {
        return kOriginKey - ((go + k * ge) << kScoreShift) - (k + 1);
    }
    static __device__ __forceinline__ T step(int64_t g) { return -((g << kScoreShift) + 1); }
    static __device__ __forceinline__ T up(T v) { return shfl_up64(v); }
    static __device__ __forceinline__ T mx(T a, T b) { return kmax(a, b); }
    static __device__ __forceinline__ T lane_value(T v, int src) { return readlane64(v, src); }
};

__host__ __device__ inline bool box32_ok(int M, int N, int go, int ge)
{
    if (M > kKey32Field || N > kKey32Field || go > 4096 || ge > 4096) return false;
    const int64_t mn = M < N ? M : N;
    // the most negative value a cell can hold (maxima, so at least the score
    // of one simple path to it) and the largest positive one, both inside
    // the 14-bit signed score field with room for one more gap step
    const int64_t low = 4 * mn + 2 * (int64_t)go + (int64_t)ge * (M + N) + go + ge;
    return low <= 8000 && 11 * mn <= 8000;
}

__host__ __device__ inline bool box64x_ok(int M, int N, int go, int ge)
{
    const int64_t mn = M < N ? M : N;
    const int64_t low = 4 * mn + 2 * (int64_t)go + (int64_t)ge * (M + N) + go + ge;
    return low <= 4000000 && 11 * mn <= 4000000;  // the score field holds +-2^23
}

// The exact sweep: the wavefront of sweep_box with keys of format K, the
// diagonal step of each (query, reference) code pair from a table in LDS,
// exact keys of leading gaps above and left of the box (every value is the
// key of a real path from the box's origin, so none is dropped) and a
// constant that loses every maximum for the states that cannot exist there
// (E left of the box, F above it).
template <int R, typename K>
__device__ __forceinline__ typename K::T sweep_box_exact(const typename K::T* step_tab, typename K::T* Hrow,
                                                         typename K::T* Frow, const uint32_t* qnib,
                                                         const uint32_t* qhib, const uint32_t* rnib,
                                                         const uint32_t* rhib, int32_t go, int32_t ge, int M, int N,
                                                         int64_t Q0, int64_t R0, int lane, bool& bad_code, int row0,
                                                         int row1)
{
    typedef typename K::T T;
    constexpr int kStrip = 64 * R;
    const T GO = K::step(go), GE = K::step(ge);
    const int n_strips = (row1 - row0 + kStrip - 1) / kStrip;
    T fin = K::kNeg;
    for (int st = 0; st < n_strips; ++st) {
        const int base = row0 + st * kStrip;
        const int rows = min(kStrip, row1 - base);
        const int i0 = base + R * lane;
        const bool ok0 = R * lane < rows;
        const T* tabr[R];
        T E[R], Hleft[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            uint32_t qc = R * lane + r < rows ? code_at(qnib, qhib, Q0 + i0 + r) : 0u;
            if (qc >= (uint32_t)kNumSym) {
                bad_code = true;
                qc = 0;
            }
            tabr[r] = step_tab + qc * kNumSym;
            E[r] = K::kNeg;                      // E left of the box cannot exist
            Hleft[r] = K::gap(go, ge, i0 + r);   // H left of the box: a leading gap of i + 1
        }
        // lane 0's first diagonal: the origin (strip 0) or the column left of the box
        T diag_next = K::kNeg;
        if (lane == 0) diag_next = base > 0 ? K::gap(go, ge, base - 1) : std::is_same<K, Key32>::value ? (T)0 : (T)kOriginKey;
        T outH = K::kNeg, outF = K::kNeg;
        uint32_t rc_prev = 0;
        uint32_t cur = code_at(rnib, rhib, R0 + lane);
        uint32_t nxt = code_at(rnib, rhib, R0 + 64 + lane);
        const bool above = base > 0;
        T curH = 0, curF = 0, nxtH = 0, nxtF = 0;
        if (above) {
            curH = Hrow[lane];
            curF = Frow[lane];
            nxtH = Hrow[min(64 + lane, kIdentMaxCols - 1)];
            nxtF = Frow[min(64 + lane, kIdentMaxCols - 1)];
        }
        const int lanes_used = (rows + R - 1) / R;
        const int steps = N + lanes_used - 1;
        for (int t = 0; t < steps; ++t) {
            if (t > 0 && (t & 63) == 0) {
                cur = nxt;
                nxt = code_at(rnib, rhib, R0 + t + 64 + lane);
                if (above) {
                    curH = nxtH;
                    curF = nxtF;
                    const int c = min(t + 64 + lane, kIdentMaxCols - 1);
                    nxtH = Hrow[c];
                    nxtF = Frow[c];
                }
            }
            const int src = t & 63;
            const uint32_t rc_new = readlane32(cur, src);
            const uint32_t rc_up = (uint32_t)__shfl_up((int)rc_prev, 1, 64);
            const uint32_t rc = lane == 0 ? rc_new : rc_up;
            rc_prev = rc;
            T upH = K::up(outH);
            T upF = K::up(outF);
            const T topH = K::lane_value(curH, src);
            const T topF = K::lane_value(curF, src);
            if (lane == 0) {
                // the row above: the previous strip's bottom row, or above
                // the box the keys of a leading gap (no F there)
                upH = above ? topH : K::gap(go, ge, t);
                upF = above ? topF : K::kNeg;
            }
            const T diag = diag_next;
            diag_next = upH;
            const int j = t - lane;
            if (ok0 && j >= 0 && j < N) {
                uint32_t rcc = rc;
                if (rcc >= (uint32_t)kNumSym) {
                    bad_code = true;
                    rcc = 0;
                }
                T dg = diag;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const T d = dg + tabr[r][rcc];
                    E[r] = K::mx(E[r] + GE, Hleft[r] + GO);
                    const T F = K::mx(upF + GE, upH + GO);
                    const T H = K::mx(d, K::mx(E[r], F));
                    dg = Hleft[r];
                    Hleft[r] = H;
                    upH = H;
                    upF = F;
                    if (j == N - 1 && i0 + r == M - 1) fin = H;
                }
                outH = upH;
                outF = upF;
                if (lane == 63 && base + kStrip < M) {  // a full strip with rows below it
                    Hrow[j] = upH;
                    Frow[j] = upF;
                }
            } else if (j == -1) {
                // the column left of the box, for the next lane's diagonal
                outH = K::gap(go, ge, i0 + R - 1);
                outF = K::kNeg;
            } else {
                outH = K::kNeg;
                outF = K::kNeg;
            }
        }
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the bottom row is in memory
    }
    return fin;
}

__global__ void __launch_bounds__(64 * kIdentWavesPerBlock, 4) k_identity(IdentArgs a)
{
    __shared__ int8_t sub[kNumSym * kNumSym];
    __shared__ int32_t step32[kNumSym * kNumSym];  // diagonal step of a 32-bit key
    __shared__ int64_t step64[kNumSym * kNumSym];  // and of a 64-bit one
    for (int i = threadIdx.x; i < kNumSym * kNumSym; i += blockDim.x) {
        sub[i] = a.subst[i];
        const int match = (i / kNumSym) == (i % kNumSym) ? 1 : 0;
        step32[i] = ((int32_t)a.subst[i] << kKey32ScoreShift) + (match << kKey32MatchShift) + 1;
        step64[i] = ((int64_t)a.subst[i] << kScoreShift) + ((int64_t)match << kMatchShift) - 1;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * kIdentWavesPerBlock + (threadIdx.x >> 6);
    int64_t* Hrow = a.scratch + wave * (2 * (int64_t)kIdentMaxCols);
    int64_t* Frow = Hrow + kIdentMaxCols;
    const uint32_t* qnib = a.qblk;
    const uint32_t* qhib = a.qblk + a.qhdr->n_blocks * 32;
    const uint32_t* rnib = a.rblk;
    const uint32_t* rhib = a.rblk + a.rhdr->n_blocks * 32;
    const int64_t q_res = a.qhdr->n_residues, r_res = a.rhdr->n_residues;
    // gap steps as keys to add: minus the cost in the score field, one column
    // more (a 64-bit add is one instruction, a subtraction two)
    const int64_t GO = -(((int64_t)a.go << kScoreShift) + 1);
    const int64_t GE = -(((int64_t)a.ge << kScoreShift) + 1);
    bool bad_range = false, bad_code = false, bad_box = false;

    for (;;) {
        int t = 0;
        if (lane == 0) t = atomicAdd(a.next_pair, 1);
        t = __shfl(t, 0, 64);
        if ((int64_t)t >= a.n_pairs) break;
        const int k = a.order[t];
        const sw_result res = a.aligned[k];
        sw_identity_result rec = {0, 0, 0, 0};
        bool ok = res.score > 0;
        int64_t qb = 0, rb = 0, m = 0, n = 0;
        if (ok) {
            const int64_t qi = a.pairs[2 * (int64_t)k], ri = a.pairs[2 * (int64_t)k + 1];
            if (qi < 0 || qi >= a.n_q || ri < 0 || ri >= a.n_r) {
                ok = false;
            } else {
                qb = a.q_offsets[qi];
                m = a.q_offsets[qi + 1] - qb;
                rb = a.r_offsets[ri];
                n = a.r_offsets[ri + 1] - rb;
                ok = qb >= 0 && m >= 0 && qb + m <= q_res && rb >= 0 && n >= 0 && rb + n <= r_res &&
                     m <= SW_MAX_SEQ_LEN && n <= SW_MAX_SEQ_LEN && res.q_start >= 0 && res.q_end >= res.q_start &&
                     res.q_end < m && res.r_start >= 0 && res.r_end >= res.r_start && res.r_end < n;
            }
            bad_range = bad_range || !ok;
        }
        if (!ok) {
            if (lane == 0) a.out[k] = rec;
            continue;
        }
        const int M = res.q_end - res.q_start + 1, N = res.r_end - res.r_start + 1;
        const bool covered = (1000 * (int64_t)M >= (int64_t)a.cov_permille * m) &&
                             (1000 * (int64_t)N >= (int64_t)a.cov_permille * n);
        if (a.coverage_first && !covered) {  // cannot be kept: no sweep
            rec.score = res.score;
            rec.matches = -1;
            rec.columns = -1;
            if (lane == 0) a.out[k] = rec;
            continue;
        }
        const int64_t Q0 = qb + res.q_start, R0 = rb + res.r_start;
        // rows per lane: 4 for every full 256-row strip, and for the box's
        // last strip the fewest (1, 2 or 4) that cover its rows -- a strip
        // costs the wave about N steps of R cells per lane whatever its height
        const int m4 = M > 256 ? (M - 1) / 256 * 256 : 0;
        const int r_last = M - m4 <= 64 ? 1 : (M - m4 <= 128 ? 2 : 4);
        const int fin_lane = (M - 1 - m4) / r_last;
        int64_t fin = kNegKey;
        if (box32_ok(M, N, a.go, a.ge)) {
            int32_t* H32 = reinterpret_cast<int32_t*>(Hrow);
            int32_t* F32 = reinterpret_cast<int32_t*>(Frow);
            int32_t f32 = Key32::kNeg;
            for (int seg = m4 > 0 ? 0 : 1; seg < 2; ++seg) {
                const int r0 = seg == 0 ? 0 : m4, r1 = seg == 0 ? m4 : M, rr = seg == 0 ? 4 : r_last;
                if (rr == 1)
                    f32 = sweep_box_exact<1, Key32>(step32, H32, F32, qnib, qhib, rnib, rhib, a.go, a.ge, M, N, Q0,
                                                    R0, lane, bad_code, r0, r1);
                else if (rr == 2)
                    f32 = sweep_box_exact<2, Key32>(step32, H32, F32, qnib, qhib, rnib, rhib, a.go, a.ge, M, N, Q0,
                                                    R0, lane, bad_code, r0, r1);
                else
                    f32 = sweep_box_exact<4, Key32>(step32, H32, F32, qnib, qhib, rnib, rhib, a.go, a.ge, M, N, Q0,
                                                    R0, lane, bad_code, r0, r1);
            }
            if (lane == fin_lane) {
                rec.score = f32 >> kKey32ScoreShift;  // arithmetic: a negative score stays negative
                rec.matches = (f32 >> kKey32MatchShift) & kKey32Field;
                rec.columns = M + N - (f32 & kKey32Field);
                if (rec.score > 0)
                    rec.keep = (1000 * (int64_t)rec.matches >= (int64_t)a.ani_permille * rec.columns) && covered;
                else
                    rec = sw_identity_result{0, 0, 0, 0};
                if (rec.score != res.score) bad_box = true;
                a.out[k] = rec;
            }
            continue;
        }
        const bool exact = box64x_ok(M, N, a.go, a.ge);
        for (int seg = m4 > 0 ? 0 : 1; seg < 2; ++seg) {
            const int r0 = seg == 0 ? 0 : m4, r1 = seg == 0 ? m4 : M, rr = seg == 0 ? 4 : r_last;
            if (exact && rr == 1)
                fin = sweep_box_exact<1, Key64>(step64, Hrow, Frow, qnib, qhib, rnib, rhib, a.go, a.ge, M, N, Q0, R0,
                                                lane, bad_code, r0, r1);
            else if (exact && rr == 2)
                fin = sweep_box_exact<2, Key64>(step64, Hrow, Frow, qnib, qhib, rnib, rhib, a.go, a.ge, M, N, Q0, R0,
                                                lane, bad_code, r0, r1);
            else if (exact)
                fin = sweep_box_exact<4, Key64>(step64, Hrow, Frow, qnib, qhib, rnib, rhib, a.go, a.ge, M, N, Q0, R0,
                                                lane, bad_code, r0, r1);
            else if (rr == 1)
                fin = sweep_box<1>(sub, Hrow, Frow, qnib, qhib, rnib, rhib, GO, GE, M, N, Q0, R0, lane, bad_code, r0,
                                   r1);
            else if (rr == 2)
                fin = sweep_box<2>(sub, Hrow, Frow, qnib, qhib, rnib, rhib, GO, GE, M, N, Q0, R0, lane, bad_code, r0,
                                   r1);
            else
                fin = sweep_box<4>(sub, Hrow, Frow, qnib, qhib, rnib, rhib, GO, GE, M, N, Q0, R0, lane, bad_code, r0,
                                   r1);
        }
        if (lane == fin_lane) {
            if ((fin >> kScoreShift) > 0) {
                rec.score = (int32_t)(fin >> kScoreShift);
                rec.matches = (int32_t)((fin >> kMatchShift) & kFieldMask);
                rec.columns = (int32_t)(kFieldMask - (fin & kFieldMask));
                rec.keep = (1000 * (int64_t)rec.matches >= (int64_t)a.ani_permille * rec.columns) && covered;
            }
            if (rec.score != res.score) bad_box = true;
            a.out[k] = rec;
        }
    }
    int bits = (bad_range || bad_box ? kErrRange : 0) | (bad_code ? kErrCode : 0);
    if (bits) atomicOr(a.err, bits);
}

}  // namespace

// Work order: a pair's tier is floor(log2) of its box cells (tier 0 up to
// 2^10 cells, the last tier from 2^24), pairs without a box in tier 0; the
// order lists the tiers from the largest down, so the long sweeps start first
// and the short ones fill the end of the launch.
__device__ __forceinline__ int box_tier(const IdentArgs& a, int64_t k)
{
    const sw_result r = a.aligned[k];
    if (r.score <= 0) return 0;
    const int64_t cells = (int64_t)(r.q_end - r.q_start + 1) * (int64_t)(r.r_end - r.r_start + 1);
    if (cells <= 1024) return 0;
    const int lg = 63 - __clzll((unsigned long long)cells);
    return min(lg - 9, kIdentTiers - 1);
}

// Counts per tier: each block counts its pairs in LDS and adds its counts
// with one global atomic per tier (an atomic per pair on 16 addresses took
// 5.6 ms for 921,422 pairs).
__global__ void __launch_bounds__(256) k_ident_count(IdentArgs a, int32_t* tiers)
{
    __shared__ int h[kIdentTiers];
    if (threadIdx.x < kIdentTiers) h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.n_pairs;
         k += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[box_tier(a, k)], 1);
    __syncthreads();
    if (threadIdx.x < kIdentTiers && h[threadIdx.x] > 0) atomicAdd(&tiers[threadIdx.x], h[threadIdx.x]);
}

// one thread: cursors start at the tier's place, largest tier first
__global__ void k_ident_offsets(int32_t* tiers)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int run = 0;
        for (int t = kIdentTiers - 1; t >= 0; --t) {
            const int c = tiers[t];
            tiers[kIdentTiers + t] = run;
            run += c;
        }
    }
}

// Places each pair in its tier's range: each block counts its pairs per
// tier in LDS, reserves its part of every tier's range with one global atomic
// per tier, then hands out places from LDS cursors (the order inside a tier
// is free).
__global__ void __launch_bounds__(256) k_ident_scatter(IdentArgs a, int32_t* tiers, int32_t* order)
{
    __shared__ int h[kIdentTiers];
    if (threadIdx.x < kIdentTiers) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t k0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = k0; k < a.n_pairs; k += stride) atomicAdd(&h[box_tier(a, k)], 1);
    __syncthreads();
    if (threadIdx.x < kIdentTiers) {
        const int c = h[threadIdx.x];
        h[threadIdx.x] = c > 0 ? atomicAdd(&tiers[kIdentTiers + threadIdx.x], c) : 0;
    }
    __syncthreads();
    for (int64_t k = k0; k < a.n_pairs; k += stride) order[atomicAdd(&h[box_tier(a, k)], 1)] = (int32_t)k;
}

__global__ void k_ident_zero(int32_t* tiers, int32_t* next_pair)
{
    if (threadIdx.x < 2 * kIdentTiers) tiers[threadIdx.x] = 0;
    if (threadIdx.x == 0) *next_pair = 0;
}

hipError_t launch_identity_order(const IdentArgs& a, int32_t* tiers, int32_t* order, hipStream_t stream)
{
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((a.n_pairs + 255) / 256, 2048));
    hipLaunchKernelGGL(k_ident_zero, dim3(1), dim3(64), 0, stream, tiers, a.next_pair);
    hipLaunchKernelGGL(k_ident_count, dim3((unsigned)blocks), dim3(256), 0, stream, a, tiers);
    hipLaunchKernelGGL(k_ident_offsets, dim3(1), dim3(64), 0, stream, tiers);
    hipLaunchKernelGGL(k_ident_scatter, dim3((unsigned)blocks), dim3(256), 0, stream, a, tiers, order);
    return hipGetLastError();
}

hipError_t launch_identity(const IdentArgs& a, int blocks, hipStream_t stream)
{
    hipLaunchKernelGGL(k_identity, dim3((unsigned)blocks), dim3(64 * kIdentWavesPerBlock), 0, stream, a);
    return hipGetLastError();
}

// The edges of the similarity graph: pairs whose identity record keeps them,
// with their alignment and identity records, appended to the output at
// *count in no particular order (one atomic per wave; slots past `cap` are
// counted, not written).
__global__ void k_edges(const int32_t* __restrict__ pairs, const sw_result* __restrict__ res,
                        const sw_identity_result* __restrict__ id, int64_t n, int32_t* __restrict__ e_pairs,
                        sw_result* __restrict__ e_res, sw_identity_result* __restrict__ e_id, int64_t cap,
                        unsigned long long* count)
{
    const int lane = threadIdx.x & 63;
    // every lane of a wave takes the same trips (the ballot needs all of them)
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = base + threadIdx.x;
        const bool keep = k < n && id[k].keep == 1;
        const unsigned long long mask = __ballot(keep);
        if (mask == 0) continue;
        const int leader = __ffsll((long long)mask) - 1;
        unsigned long long first = 0;
        if (lane == leader) first = atomicAdd(count, (unsigned long long)__popcll(mask));
        first = __shfl(first, leader, 64);
        if (keep) {
            const int64_t slot = (int64_t)(first + (unsigned long long)__popcll(mask & ((1ull << lane) - 1)));
            if (slot < cap) {
                e_pairs[2 * slot] = pairs[2 * k];
                e_pairs[2 * slot + 1] = pairs[2 * k + 1];
                e_res[slot] = res[k];
                e_id[slot] = id[k];
            }
        }
    }
}

hipError_t launch_edges(const int32_t* pairs, const sw_result* res, const sw_identity_result* id, int64_t n,
                        int32_t* e_pairs, sw_result* e_res, sw_identity_result* e_id, int64_t cap,
                        unsigned long long* count, hipStream_t stream)
{
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    if (blocks > 0)
        hipLaunchKernelGGL(k_edges, dim3((unsigned)blocks), dim3(256), 0, stream, pairs, res, id, n, e_pairs, e_res,
                           e_id, cap, count);
    return hipGetLastError();
}

}  // namespace swk
