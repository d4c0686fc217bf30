// Set-up primitives of the plan (bs_prim.hip): deterministic integer scan
// and stable radix sort, asynchronous on `st` except that each synchronises
// before freeing its own temporaries.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bs.h"

namespace bs {

// out[i] = in[0] + ... + in[i-1] for 0 <= i < n (int32 counts whose total
// stays below 2^31); in and out may be the same array.
bs_status scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t st, const char* op);

// Stable sort of n (key, value) pairs by the low `bits` bits of the keys,
// ascending; equal keys keep their input order.  keys/vals hold the input
// and keys_alt/vals_alt are scratch of the same sizes; the sorted pairs end
// in keys_alt/vals_alt when *in_alt is set, else in keys/vals.
bs_status sort_pairs_u32(uint32_t* keys, uint32_t* keys_alt, int32_t* vals, int32_t* vals_alt, int64_t n, int bits,
                         hipStream_t st, const char* op, bool* in_alt);

}  // namespace bs
