// Internal declarations of the identity / coverage pass (sw_identity.hip),
// used by the host layer (sw_api.cpp).  Not part of the public interface.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "sw_internal.h"

namespace swk {

constexpr int kIdentMaxCols = SW_MAX_SEQ_LEN + 1;  // scratch columns per wave (a box is at most this wide)
constexpr int kIdentWavesPerBlock = 4;

struct IdentArgs {
    const uint32_t* qblk;
    const PackedHeader* qhdr;
    const int64_t* q_offsets;
    int64_t n_q;
    const uint32_t* rblk;
    const PackedHeader* rhdr;
    const int64_t* r_offsets;
    int64_t n_r;
    const int32_t* pairs;
    int64_t n_pairs;
    const sw_result* aligned;
    sw_identity_result* out;
    const int8_t* subst;    // [24 * 24] scores in the packed code order
    int64_t* scratch;       // per wave: kIdentMaxCols H keys, then kIdentMaxCols F keys
    int32_t* next_pair;     // work counter (zero before the launch)
    const int32_t* order;   // [n_pairs] pair indices, largest boxes first (launch_identity_order)
    int32_t* err;           // device error bits (kErr*)
    int32_t go, ge;
    int32_t ani_permille, cov_permille;
    int32_t coverage_first;  // skip pairs whose coverage fails
};

hipError_t launch_identity(const IdentArgs& a, int blocks, hipStream_t stream);
// the work order of the pass: pairs by tier of box cells, largest first
// (tiers[] holds kIdentTiers counts and as many cursors; order[] n_pairs)
constexpr int kIdentTiers = 16;
hipError_t launch_identity_order(const IdentArgs& a, int32_t* tiers, int32_t* order, hipStream_t stream);
// the kept pairs (keep == 1) with their records, appended at *count
hipError_t launch_edges(const int32_t* pairs, const sw_result* res, const sw_identity_result* id, int64_t n,
                        int32_t* e_pairs, sw_result* e_res, sw_identity_result* e_id, int64_t cap,
                        unsigned long long* count, hipStream_t stream);

}  // namespace swk
