// Device-wide primitives used by ingest, composition and selection:
// exclusive scan of int32/int64 counts and a stable LSD radix sort of
// 64-bit keys with int32 values.  Host-side launchers; the kernels live in
// hln_prim.hip.
#pragma once

#include "hln_internal.hpp"

namespace hln {
namespace prim {

// Scratch bytes for scan_exclusive over `count` elements.
size_t scan_workspace(long long count);
// out[i] = sum_{j<i} in[i] for i <= count (out has count+1 entries; out[count]
// is the total).  in and out may alias.  T = int32_t or int64_t.
template <typename T>
hln_status scan_exclusive(const T* in, T* out, long long count, void* ws, size_t ws_bytes, hipStream_t st);

// Scratch bytes for sort_pairs over `count` elements.
size_t sort_workspace(long long count);
// Stable ascending sort of (keys, vals) by the key bits [0, key_bits) --
// higher bits must be zero.  Results land back in keys / vals.
hln_status sort_pairs(unsigned long long* keys, int32_t* vals, long long count, int key_bits, void* ws,
                      size_t ws_bytes, hipStream_t st);

}  // namespace prim
}  // namespace hln
