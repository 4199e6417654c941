// Internal declarations of candidate discovery (sw_kmer.hip), used by the
// host layer (sw_api.cpp).  Not part of the public interface.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "sw_internal.h"

namespace swk {

// One packed sequence set as the discovery kernels read it.
struct KmerSide {
    const uint32_t* blk;        // first block of the packed buffer
    const PackedHeader* hdr;
    const int64_t* offs;        // [n + 1] residue offsets
    int64_t n;
};

constexpr int kKmerMaxK = 6;              // (sequence << 32 | k-mer) keys: k-mer < 2^32
constexpr int kKmerAlphabet = 24;         // a k-mer is the base-24 number of its codes
constexpr uint64_t kEmptyKey = ~0ull;     // free slot of a hash table (all bytes 0xFF)

// 64-bit counters of one discovery call
enum {
    kKmPosR = 0,      // k-mer windows of the reference set
    kKmPosQ = 1,      // k-mer windows of the query set
    kKmProducts = 2,  // sum over query entries of the reference-list length
    kKmOut = 3,       // pairs at or above the threshold
    kKmErr = 4,       // error bits (kErr*)
    kKmNumCounters = 8
};

int64_t kmer_space(int k);  // 24^k

// all asynchronous on `stream`
hipError_t launch_kmer_positions(const KmerSide& s, int k, int slot, uint64_t* counters, hipStream_t stream);
hipError_t launch_kmer_insert(const KmerSide& s, int k, uint64_t* set, int64_t set_cap, int32_t* kcount,
                              uint64_t* counters, hipStream_t stream);
hipError_t launch_kmer_scan(int32_t* kcount, int32_t* kstart, int64_t n, int64_t* tile_sums, hipStream_t stream);
int64_t kmer_scan_tiles(int64_t n);
hipError_t launch_kmer_scatter(const uint64_t* set, int64_t set_cap, const int32_t* kstart, int32_t* kcount,
                               int32_t* rlist, hipStream_t stream);
hipError_t launch_kmer_products(const uint64_t* set, int64_t set_cap, const int32_t* kstart, uint64_t* counters,
                                hipStream_t stream);
hipError_t launch_kmer_query_products(const uint64_t* set, int64_t set_cap, const int32_t* kstart, uint64_t* qprod,
                                      hipStream_t stream);
// joins only the query entries with q_lo <= q < q_hi
hipError_t launch_kmer_join(const uint64_t* qset, int64_t qset_cap, const int32_t* kstart, const int32_t* rlist,
                            int mode, int64_t q_lo, int64_t q_hi, uint64_t* pkeys, int32_t* pcount, int64_t pcap,
                            uint64_t* counters, hipStream_t stream);
hipError_t launch_kmer_compact(const uint64_t* pkeys, const int32_t* pcount, int64_t pcap, int min_shared,
                               int32_t* pairs_out, int32_t* shared_out, int64_t out_cap, uint64_t* counters,
                               hipStream_t stream);

}  // namespace swk
