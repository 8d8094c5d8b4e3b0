// Device-wide primitives used by ingest, composition and selection:
// exclusive scan of int32/int64 counts and a stable LSD radix sort of
// 64-bit keys with int32 values, over a whole array or over many segments
// at once.  Host-side launchers; the kernels live in
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

// Segmented stable sort of 64-bit keys, with int32 values moving along when
// vals (and valt) are given: segment s is keys [key_off[s], key_off[s+1])
// and is sorted on its own by the key bits [0, key_bits).  key_off and
// tile_off are device arrays of nseg + 1 entries; tile_off[s+1] -
// tile_off[s] = seg_sort_tiles(segment length) and tiles = tile_off[nseg].
// The sorted keys (values) end in keys (vals), or in alt (valt) when
// *in_alt is set on return.
long long seg_sort_tiles(long long count);
size_t seg_sort_workspace(long long tiles);
hln_status sort_segmented(unsigned long long* keys, unsigned long long* alt, int32_t* vals, int32_t* valt,
                          const long long* key_off, const long long* tile_off, int nseg, long long tiles, int key_bits,
                          void* ws, size_t ws_bytes, hipStream_t st, bool* in_alt);

}  // namespace prim
}  // namespace hln
