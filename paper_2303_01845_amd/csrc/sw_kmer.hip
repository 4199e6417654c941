// Candidate discovery on the GPU: which (query, reference) pairs have at
// least `min_shared` distinct k-mers in common.
//
// The paper (section "Protein similarity search pipeline") forms the
// sequence-by-k-mer matrix A, whose nonzero (s, x) marks that k-mer x occurs
// in sequence s, and finds candidates through an overloaded sparse product
// C = A_q A_r^T that counts common k-mers; a pair is aligned when its count
// reaches the common k-mer threshold (k = 6, threshold 2 in the program
// parameters of section "Similarity search at scale").  Self searches keep one
// of C[i][j], C[j][i] (section "Load balancing techniques").
//
// The GPU form of that product, with no floating-point SpGEMM in sight:
//   1. positions: count the k-mer windows of each set, and check its offsets;
//   2. insert: every window's (sequence << 32 | k-mer) key goes into an
//      open-addressing hash set, which leaves each nonzero of A once (a
//      sequence that repeats a k-mer still holds it once);
//   3. index: the reference entries are counting-sorted by k-mer over the
//      dense space of 24^k k-mers (a histogram built during the insert, an
//      exclusive scan, a scatter), giving the columns of A_r as lists;
//   4. join: every query entry (q, x) walks the reference list of x and adds
//      one to the (q, r) counter of a second hash table -- the semiring sum
//      (under a memory budget, one pass per range of queries, each with its
//      own table: the product formed block by block);
//   5. compact: counters at or above the threshold are written out.
// Every hash probe loop stops after `capacity` probes; tables are sized at
// least twice their largest possible occupancy, so a probe sequence always
// meets a free slot well before that.
#include <algorithm>

#include "kmer_internal.h"

namespace swk {

namespace {

// MurmurHash3's 64-bit finaliser (Appleby): a full-avalanche mix of the key.
__device__ __forceinline__ uint64_t mix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

// Code of the residue at position `pos` of a packed buffer (see the packed
// format: nibble plane, then the high plane after 32 n_blocks words).
__device__ __forceinline__ uint32_t code_at(const uint32_t* __restrict__ nib, const uint32_t* __restrict__ hib,
                                            int64_t pos)
{
    const int64_t q = pos + kGuardRes;
    const uint32_t lo = (nib[q >> 3] >> (4 * (uint32_t)(q & 7))) & 15u;
    const uint32_t hi = (hib[q >> 5] >> (uint32_t)(q & 31)) & 1u;
    return lo | (hi << 4);
}

__device__ __forceinline__ void set_err(uint64_t* counters, uint64_t bits)
{
    atomicOr((unsigned long long*)&counters[kKmErr], (unsigned long long)bits);
}

// Sum of a wave's values on every lane.
__device__ __forceinline__ uint64_t wave_sum(uint64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------- 1. positions
__global__ void k_positions(KmerSide s, int k, int slot, uint64_t* counters)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const PackedHeader* h = s.hdr;
    const bool hdr_ok = h->magic == kPackMagic && h->n_residues >= 0;
    const int64_t n_res = hdr_ok ? h->n_residues : 0;
    uint64_t cnt = 0;
    bool bad = !hdr_ok;
    for (int64_t i = tid; i < s.n; i += stride) {
        const int64_t a = s.offs[i], b = s.offs[i + 1];
        if (a < 0 || b < a || b > n_res) {
            bad = true;
            continue;
        }
        if (b - a >= k) cnt += (uint64_t)(b - a - k + 1);
    }
    cnt = wave_sum(cnt);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd((unsigned long long*)&counters[slot], (unsigned long long)cnt);
    if (bad) set_err(counters, kErrRange);
}

// ---------------------------------------------------------------- 2. insert
// One wave per sequence (grid-stride over sequences).  A wave covers 64
// windows at a time: lane l loads the codes at window offsets l and l + 64,
// and window l takes its k codes from lanes l .. l+k-1 of that 128-code
// stretch through lane shuffles, so each code is loaded twice per wave
// instead of k times per window.
__global__ void __launch_bounds__(256) k_insert(KmerSide s, int k, uint64_t* __restrict__ set, uint64_t mask,
                                                int32_t* __restrict__ kcount, uint64_t* counters)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const uint32_t* nib = s.blk;
    const uint32_t* hib = s.blk + s.hdr->n_blocks * 32;
    bool bad_code = false, full = false;
    for (int64_t seq = wave; seq < s.n; seq += n_waves) {
        const int64_t base = s.offs[seq];
        const int64_t L = s.offs[seq + 1] - base;
        for (int64_t p0 = 0; p0 + k <= L; p0 += 64) {
            // codes beyond the sequence read the buffer's padding: in bounds,
            // and never part of a window that is used
            const uint32_t c0 = code_at(nib, hib, base + p0 + lane);
            const uint32_t c1 = code_at(nib, hib, base + p0 + 64 + lane);
            uint32_t x = 0;
            bool ok = true;
            for (int t = 0; t < k; ++t) {
                const int src = lane + t;  // 0 .. 68
                const uint32_t a = (uint32_t)__shfl((int)c0, src & 63, 64);
                const uint32_t b = (uint32_t)__shfl((int)c1, src & 63, 64);
                const uint32_t c = src < 64 ? a : b;
                ok = ok && c < (uint32_t)kKmerAlphabet;
                x = x * (uint32_t)kKmerAlphabet + (c < (uint32_t)kKmerAlphabet ? c : 0u);
            }
            const int64_t p = p0 + lane;
            if (p + k > L) continue;
            if (!ok) {
                bad_code = true;
                continue;
            }
            const uint64_t key = ((uint64_t)seq << 32) | x;
            uint64_t h = mix64(key) & mask;
            bool placed = false;
            for (uint64_t probe = 0; probe <= mask; ++probe) {
                const uint64_t old = atomicCAS((unsigned long long*)&set[h], (unsigned long long)kEmptyKey,
                                               (unsigned long long)key);
                if (old == kEmptyKey) {  // first time this sequence shows this k-mer
                    if (kcount) atomicAdd(&kcount[x], 1);
                    placed = true;
                    break;
                }
                if (old == key) {  // a repeat within the sequence
                    placed = true;
                    break;
                }
                h = (h + 1) & mask;
            }
            full = full || !placed;
        }
    }
    if (bad_code) set_err(counters, kErrCode);
    if (full) set_err(counters, kErrInternal);
}

// ---------------------------------------------------------------- 3. index
// Exclusive scan of the per-k-mer counts over the dense k-mer space, in three
// launches: per-tile totals, a scan of the totals, and the per-tile scan that
// writes the starts (and clears the counts, which the scatter reuses as fill
// cursors).  A tile is 16 rounds of 256 consecutive counts; thread t takes
// element t of each round, so every load and store is coalesced.
constexpr int kScanThreads = 256;
constexpr int kScanRounds = 16;
constexpr int kScanTile = kScanThreads * kScanRounds;

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t* total)
{
    __shared__ int64_t wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / 64; ++i) {
        before += i < w ? wsum[i] : 0;
        all += wsum[i];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

// Sum over the block, returned on every thread.
__device__ __forceinline__ int64_t block_sum(int64_t v)
{
    __shared__ int64_t wsum[kScanThreads / 64];
    v = (int64_t)wave_sum((uint64_t)v);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t all = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / 64; ++i) all += wsum[i];
    __syncthreads();
    return all;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const int32_t* __restrict__ kcount, int64_t n,
                                                             int64_t* __restrict__ tile_sums)
{
    const int64_t first = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
    int64_t s = 0;
#pragma unroll 4
    for (int r = 0; r < kScanRounds; ++r) {
        const int64_t i = first + (int64_t)r * kScanThreads;
        if (i < n) s += kcount[i];
    }
    const int64_t total = block_sum(s);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// One block: exclusive scan of the tile totals in place; the grand total goes
// to kstart[n].
__global__ void __launch_bounds__(kScanThreads) k_scan_totals(int64_t* tile_sums, int64_t n_tiles,
                                                              int32_t* kstart, int64_t n)
{
    int64_t carry = 0;
    for (int64_t b = 0; b < n_tiles; b += kScanThreads) {
        const int64_t i = b + threadIdx.x;
        const int64_t v = i < n_tiles ? tile_sums[i] : 0;
        int64_t total;
        const int64_t ex = block_exclusive_scan(v, &total);
        if (i < n_tiles) tile_sums[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) kstart[n] = (int32_t)carry;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(int32_t* __restrict__ kcount, int64_t n,
                                                             const int64_t* __restrict__ tile_sums,
                                                             int32_t* __restrict__ kstart)
{
    const int64_t first = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
    int32_t v[kScanRounds];
#pragma unroll
    for (int r = 0; r < kScanRounds; ++r) {
        const int64_t i = first + (int64_t)r * kScanThreads;
        v[r] = i < n ? kcount[i] : 0;
    }
    int64_t run = tile_sums[blockIdx.x];
#pragma unroll
    for (int r = 0; r < kScanRounds; ++r) {
        const int64_t i = first + (int64_t)r * kScanThreads;
        int64_t total;
        const int64_t ex = block_exclusive_scan(v[r], &total);
        if (i < n) {
            kstart[i] = (int32_t)(run + ex);
            kcount[i] = 0;
        }
        run += total;
    }
}

__global__ void k_scatter(const uint64_t* __restrict__ set, int64_t cap, const int32_t* __restrict__ kstart,
                          int32_t* __restrict__ kcount, int32_t* __restrict__ rlist)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += stride) {
        const uint64_t key = set[i];
        if (key == kEmptyKey) continue;
        const uint32_t x = (uint32_t)key;
        const int32_t at = kstart[x] + atomicAdd(&kcount[x], 1);
        rlist[at] = (int32_t)(key >> 32);
    }
}

// ---------------------------------------------------------------- 4. join
// Grid-stride over the query entries with a fixed grid: one atomic per block.
__global__ void __launch_bounds__(kScanThreads) k_products(const uint64_t* __restrict__ set, int64_t cap,
                                                           const int32_t* __restrict__ kstart, uint64_t* counters)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t s = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += stride) {
        const uint64_t key = set[i];
        if (key == kEmptyKey) continue;
        const uint32_t x = (uint32_t)key;
        s += kstart[x + 1] - kstart[x];
    }
    s = block_sum(s);
    if (threadIdx.x == 0 && s) atomicAdd((unsigned long long*)&counters[kKmProducts], (unsigned long long)s);
}

// Per-query number of k-mer matches (for splitting the join into query
// ranges whose pair tables fit a memory budget).
__global__ void k_query_products(const uint64_t* __restrict__ set, int64_t cap, const int32_t* __restrict__ kstart,
                                 uint64_t* __restrict__ qprod)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += stride) {
        const uint64_t key = set[i];
        if (key == kEmptyKey) continue;
        const uint32_t x = (uint32_t)key;
        const int32_t len = kstart[x + 1] - kstart[x];
        if (len > 0) atomicAdd((unsigned long long*)&qprod[key >> 32], (unsigned long long)len);
    }
}

// Pair filter of a self search: 0 keeps all, 1 the strict upper triangle,
// 2 the index-parity rule (below the diagonal equal parities, above it
// different ones).
__device__ __forceinline__ bool keep_pair(uint32_t q, uint32_t r, int mode)
{
    if (mode == 0) return true;
    if (q == r) return false;
    if (mode == 1) return q < r;
    return (q > r) == (((q ^ r) & 1u) == 0u);
}

__global__ void k_join(const uint64_t* __restrict__ qset, int64_t qcap, const int32_t* __restrict__ kstart,
                       const int32_t* __restrict__ rlist, int mode, uint32_t q_lo, uint32_t q_hi,
                       uint64_t* __restrict__ pkeys, int32_t* __restrict__ pcount, uint64_t pmask,
                       uint64_t* counters)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool full = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < qcap; i += stride) {
        const uint64_t key = qset[i];
        if (key == kEmptyKey) continue;
        const uint32_t q = (uint32_t)(key >> 32), x = (uint32_t)key;
        if (q < q_lo || q >= q_hi) continue;  // another query range's pass
        const int32_t lo = kstart[x], hi = kstart[x + 1];
        for (int32_t e = lo; e < hi; ++e) {
            const uint32_t r = (uint32_t)rlist[e];
            if (!keep_pair(q, r, mode)) continue;
            const uint64_t pk = ((uint64_t)q << 32) | r;
            uint64_t h = mix64(pk) & pmask;
            bool placed = false;
            for (uint64_t probe = 0; probe <= pmask; ++probe) {
                uint64_t cur = pkeys[h];
                if (cur == kEmptyKey)
                    cur = atomicCAS((unsigned long long*)&pkeys[h], (unsigned long long)kEmptyKey,
                                    (unsigned long long)pk);
                if (cur == kEmptyKey || cur == pk) {
                    atomicAdd(&pcount[h], 1);
                    placed = true;
                    break;
                }
                h = (h + 1) & pmask;
            }
            full = full || !placed;
        }
    }
    if (full) set_err(counters, kErrInternal);
}

// ---------------------------------------------------------------- 5. compact
// Each wave owns a segment of kCompactSeg consecutive slots: it counts its
// hits, reserves that many output places with one atomic, then writes them in
// slot order.  (One atomic per wave and 64 slots made that single counter the
// bottleneck.)
constexpr int kCompactRounds = 32;
constexpr int kCompactSeg = 64 * kCompactRounds;

__global__ void __launch_bounds__(256) k_compact(const uint64_t* __restrict__ pkeys,
                                                 const int32_t* __restrict__ pcount, int64_t pcap, int min_shared,
                                                 int32_t* __restrict__ pairs_out, int32_t* __restrict__ shared_out,
                                                 int64_t out_cap, uint64_t* counters)
{
    const int lane = threadIdx.x & 63;
    const int64_t seg = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t first = seg * kCompactSeg + lane;
    uint32_t hits = 0;
    for (int r = 0; r < kCompactRounds; ++r) {
        const int64_t i = first + (int64_t)r * 64;
        const bool hit = i < pcap && pkeys[i] != kEmptyKey && pcount[i] >= min_shared;
        hits += (uint32_t)__popcll(__ballot(hit));
    }
    if (hits == 0) return;  // wave-uniform
    uint64_t base = 0;
    if (lane == 0) base = atomicAdd((unsigned long long*)&counters[kKmOut], (unsigned long long)hits);
    base = __shfl(base, 0, 64);
    for (int r = 0; r < kCompactRounds; ++r) {
        const int64_t i = first + (int64_t)r * 64;
        uint64_t key = kEmptyKey;
        int32_t c = 0;
        if (i < pcap) {
            key = pkeys[i];
            c = pcount[i];
        }
        const bool hit = key != kEmptyKey && c >= min_shared;
        const uint64_t m = __ballot(hit);
        if (hit) {
            const uint64_t at = base + __popcll(m & ((1ull << lane) - 1ull));
            if (at < (uint64_t)out_cap) {
                pairs_out[2 * at] = (int32_t)(key >> 32);
                pairs_out[2 * at + 1] = (int32_t)(uint32_t)key;
                if (shared_out) shared_out[at] = c;
            }
        }
        base += __popcll(m);
    }
}

unsigned grid_for(int64_t items, int threads, int64_t max_blocks = 1 << 16)
{
    const int64_t b = (items + threads - 1) / threads;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, max_blocks));
}

}  // namespace

int64_t kmer_space(int k)
{
    int64_t v = 1;
    for (int i = 0; i < k; ++i) v *= kKmerAlphabet;
    return v;
}

int64_t kmer_scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

hipError_t launch_kmer_positions(const KmerSide& s, int k, int slot, uint64_t* counters, hipStream_t stream)
{
    hipLaunchKernelGGL(k_positions, dim3(grid_for(s.n, 256, 4096)), dim3(256), 0, stream, s, k, slot, counters);
    return hipGetLastError();
}

hipError_t launch_kmer_insert(const KmerSide& s, int k, uint64_t* set, int64_t set_cap, int32_t* kcount,
                              uint64_t* counters, hipStream_t stream)
{
    // four waves per block, one sequence per wave at a time
    hipLaunchKernelGGL(k_insert, dim3(grid_for(s.n, 4, 1 << 15)), dim3(256), 0, stream, s, k, set,
                       (uint64_t)(set_cap - 1), kcount, counters);
    return hipGetLastError();
}

hipError_t launch_kmer_scan(int32_t* kcount, int32_t* kstart, int64_t n, int64_t* tile_sums, hipStream_t stream)
{
    const int64_t tiles = kmer_scan_tiles(n);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kScanThreads), 0, stream, kcount, n, tile_sums);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanThreads), 0, stream, tile_sums, tiles, kstart, n);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)tiles), dim3(kScanThreads), 0, stream, kcount, n, tile_sums,
                       kstart);
    return hipGetLastError();
}

hipError_t launch_kmer_scatter(const uint64_t* set, int64_t set_cap, const int32_t* kstart, int32_t* kcount,
                               int32_t* rlist, hipStream_t stream)
{
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(set_cap, 256)), dim3(256), 0, stream, set, set_cap, kstart, kcount,
                       rlist);
    return hipGetLastError();
}

hipError_t launch_kmer_products(const uint64_t* set, int64_t set_cap, const int32_t* kstart, uint64_t* counters,
                                hipStream_t stream)
{
    hipLaunchKernelGGL(k_products, dim3(grid_for(set_cap, 256, 2048)), dim3(256), 0, stream, set, set_cap, kstart,
                       counters);
    return hipGetLastError();
}

hipError_t launch_kmer_query_products(const uint64_t* set, int64_t set_cap, const int32_t* kstart, uint64_t* qprod,
                                      hipStream_t stream)
{
    hipLaunchKernelGGL(k_query_products, dim3(grid_for(set_cap, 256)), dim3(256), 0, stream, set, set_cap, kstart,
                       qprod);
    return hipGetLastError();
}

hipError_t launch_kmer_join(const uint64_t* qset, int64_t qset_cap, const int32_t* kstart, const int32_t* rlist,
                            int mode, int64_t q_lo, int64_t q_hi, uint64_t* pkeys, int32_t* pcount, int64_t pcap,
                            uint64_t* counters, hipStream_t stream)
{
    hipLaunchKernelGGL(k_join, dim3(grid_for(qset_cap, 256)), dim3(256), 0, stream, qset, qset_cap, kstart, rlist,
                       mode, (uint32_t)q_lo, (uint32_t)q_hi, pkeys, pcount, (uint64_t)(pcap - 1), counters);
    return hipGetLastError();
}

hipError_t launch_kmer_compact(const uint64_t* pkeys, const int32_t* pcount, int64_t pcap, int min_shared,
                               int32_t* pairs_out, int32_t* shared_out, int64_t out_cap, uint64_t* counters,
                               hipStream_t stream)
{
    // four waves per block, one segment per wave
    const int64_t segs = (pcap + kCompactSeg - 1) / kCompactSeg;
    hipLaunchKernelGGL(k_compact, dim3((unsigned)((segs + 3) / 4)), dim3(256), 0, stream, pkeys, pcount, pcap,
                       min_shared, pairs_out, shared_out, out_cap, counters);
    return hipGetLastError();
}

}  // namespace swk
