// Internal declarations shared by the device code (sw_device.hip) and the
// host layer (sw_api.cpp).  Not part of the public interface.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "../../include/sw.h"

namespace swk {

// ---------------------------------------------------------------- packed format
// A packed buffer is a 256-byte header followed by two planes over residue
// positions p in [-kGuardRes, 256 n_blocks - kGuardRes):
//   nibble plane (32 n_blocks words): residue q = p + kGuardRes in bits
//     4*(q&7).. of word q>>3
//   high plane (8 n_blocks words, right after): bit q&31 of word q>>5
// code = nibble | high << 4, in the library's own symbol order.  Each plane is
// contiguous, so a run of residues is a run of words: a lane can fetch 32
// residues with one 16-byte load.  The guard of kGuardRes residues before
// position 0 and the slack after the last residue keep every window of a few
// dozen residues that overlaps a sequence inside the buffer.  The aligner
// finds the high plane from n_blocks in the header.
constexpr uint32_t kPackMagic = 0x35575350u;  // "PSW5"
constexpr int kGuardRes = 64;
constexpr int kTailRes = 512;
constexpr int kHeaderBytes = 256;
constexpr int kNumSym = 24;
constexpr int kPadCode = 24;  // beyond a sequence end (and invalid letters); scores -4 against everything
constexpr int kNumCodes = 25;

struct PackedHeader {
    uint32_t magic;
    uint32_t version;
    int64_t n_residues;
    int64_t n_blocks;
    int64_t total_bytes;
};

inline int64_t packed_blocks(int64_t n) { return (kGuardRes + n + kTailRes + 255) / 256 + 1; }
inline size_t packed_bytes(int64_t n) { return (size_t)kHeaderBytes + (size_t)packed_blocks(n) * 160; }

// ---------------------------------------------------------------- work layout
constexpr int kWave = 64;
constexpr int kMaxInterStrips = 64;    // ceil(inter_max_len / rows_per_lane) <= this
constexpr int kMaxInterChunks = 128;   // ceil(inter_max_len / 8) <= this
constexpr int kMaxInterLen = 1024;
constexpr int kMaxP16Len = 4096;      // longest pair a 16-lane group may get; the packed
                                      // 16-bit pass also covers whole waves up to this
constexpr int kDefaultGroup16Max = 2048;  // default group16_max_len (no 16-lane groups next to the 8-lane default)
constexpr int kDefaultGroup8Max = 2048;   // default group8_max_len
constexpr int kXbufBytes = 64 * 96;   // LDS exchange / staging buffer: 24 words per lane
constexpr int kWideCostBins = 512;     // floor(16 * log2(m*n)) for long (wide) pairs
constexpr int kNumLenBuckets = 17;     // ceil(log2(max(m, n))), 0..16
constexpr int kInterCells = kMaxInterStrips * kMaxInterChunks;
constexpr int kWideCells = kNumLenBuckets * kWideCostBins;
constexpr int kNumCells = kInterCells + kWideCells;
// Each cell's count is split over this many counters (by the classify
// tile of the pair, mod kCellShards), so that the atomics of a popular cell
// do not all land on one address.
constexpr int kCellShards = 16;

// The scan of the cell counts runs over tiles of kScanRanks ranks, one block
// each, then applies every tile's prefix.
constexpr int kScanRanks = 1024;
constexpr int kScanTiles = (kNumCells + kScanRanks - 1) / kScanRanks;

// counters[] slots in the workspace
enum {
    kCntHead = 0,   // persistent work-queue head
    kCntP64 = 1,    // pairs aligned by 64 lanes (longest)
    kCntP16 = 2,    // pairs aligned by 16 lanes
    kCntP1 = 3,     // pairs aligned by one lane
    kCntP8 = 4,     // pairs aligned by 8 lanes
    kCntTiles = 16, // per scan tile: its pairs, and those of 64, 16 and 8 lanes
    kNumCounters = kCntTiles + 4 * kScanTiles
};
enum { kErrRange = 1, kErrCode = 2, kErrInternal = 4 };

struct Args {
    const uint32_t* qblk;      // first block of the query set's packed buffer
    const PackedHeader* qhdr;  // its header
    const int64_t* q_offsets;
    int64_t n_q;
    const uint32_t* rblk;      // the same for the reference set (may alias the query set)
    const PackedHeader* rhdr;
    const int64_t* r_offsets;
    int64_t n_r;
    const int32_t* pairs;
    int64_t n_pairs;
    sw_result* out;
    int32_t* pair_cell;        // [n_pairs] work cell of each pair (-1 none, -2 invalid)
    int32_t* pair_rank;        // [n_pairs] its place among the pairs of its cell and shard
    int32_t* perm;             // [n_pairs] pair indices sorted by rank of their cell
    int32_t* cell_count;       // [kNumCells][kCellShards] histogram, then first perm position
    const int32_t* rank_cell;  // [kNumCells] cell at each rank
    int32_t* rank_start;       // [kNumCells + 1] first perm position of each rank
    int32_t* counters;         // [kNumCounters]
    int32_t* err;              // device error bits of this device (kErr*)
    uint32_t* scratch;         // boundary rows, one slot per resident block
    int64_t slot_words;        // 32-bit words per slot
    int32_t go, ge;
    int32_t rows_per_lane;
    int32_t inter_max_len;
    int32_t group16_max_len;   // longest pair of a 16-lane group (power of two)
    int32_t group8_max_len;    // longest pair of an 8-lane group (power of two, <= group16_max_len)
    int32_t phase;             // 0: both passes per item; 1: forward pass only (writes score
                               // and end); 2: start pass only (reads them from out)
    int8_t bucket_kind[kNumLenBuckets];  // lanes per pair of each length bucket, 0: the rule
};
static_assert(kNumLenBuckets == SW_NUM_BUCKETS, "one override per length bucket");

// Lanes per pair of the pairs of a length bucket that do not get one lane
// each: the bucket's override if it names a group, else the threshold rule
// (8-lane groups up to group8_max, 16-lane up to group16_max, both capped at
// kMaxP16Len, a whole wave beyond).  Shared by the host's ordering and the
// device's cell bookkeeping so that both agree on every cell.
__host__ __device__ inline int bucket_group_kind(int bucket, int override_kind, int group8_max, int group16_max)
{
    if (override_kind > 1) return override_kind;
    const int len = 1 << bucket;
    const int g8 = group8_max < kMaxP16Len ? group8_max : kMaxP16Len;
    const int g16 = group16_max < kMaxP16Len ? group16_max : kMaxP16Len;
    return len <= g8 ? 8 : len <= g16 ? 16 : 64;
}

// launchers (sw_device.hip); all asynchronous on `stream`
hipError_t launch_pack(const char* ascii, int64_t n, void* packed, int32_t* err, hipStream_t stream);
hipError_t launch_prepare(const Args& a, hipStream_t stream);  // zero, classify, scan, scatter
hipError_t launch_persistent(const Args& a, int grid, hipStream_t stream);
hipError_t launch_plain(const Args& a, int kind, int first, int count, int grid, hipStream_t stream);
hipError_t set_kernel_attributes();
size_t lds_bytes(int rows_per_lane);
// 32-bit words of a block's boundary-row slot: slot_words() is the least that
// serves every kind of work item (pairs too long for three whole-wave
// buffers then sweep in place); slot_words_for(len) also gives every pair up
// to len reference residues the whole-wave scan (three buffers).
int64_t slot_words();
int64_t slot_words_for(int64_t max_len);

// Per-device state held in file-scope device arrays of sw_device.hip (no
// allocation): the two rank -> cell orderings and the error word.
// device_statics() looks their addresses up on the current device
// (hipGetSymbolAddress); each device has its own copy of every array.
struct DeviceStatics {
    int32_t* rank_cell_persistent;
    int32_t* rank_cell_plain;
    int32_t* err;
    void* static_ws;  // kStaticWsBytes, the workspace of sw_align_sets_static
};
// The fixed workspace of the allocation-free entry point and the most pairs
// one of its calls takes (their sort arrays, 32 MiB, leave room for 281
// boundary-row slots of 1,280 KiB).
constexpr size_t kStaticWsBytes = (size_t)384 << 20;
constexpr int64_t kStaticMaxPairs = (int64_t)1 << 22;
hipError_t device_statics(DeviceStatics* out);
void matrix_ncbi(int8_t out[kNumSym * kNumSym], char letters[kNumSym + 1]);
const char* code_order();

}  // namespace swk
