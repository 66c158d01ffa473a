// Internal declarations of the LBVH builder (bvh.hip), used by the host
// runtime.
#pragma once

#include "rtmc_internal.h"

namespace rtmc {

// BVH builder pieces
constexpr int kRefitLevels = 256;  // node heights the bottom-up refit can reach

struct BvhBuild {
  const float4* tris_in;  // [3 n] unsorted, compacted
  float4* tris_out;       // [3 n] sorted
  float4* tris_rot;       // [4 n] sorted, rotated records
  float4* nodes;          // [4 max(n - 1, 1)] binary nodes
  float4* nodes4;         // [4 max(n - 1, 1)] quantized 4-wide nodes (traversal)
  uint64_t* keys;         // [n]
  uint32_t* vals;         // [n]
  uint64_t* keys_alt;     // [n]
  uint32_t* vals_alt;     // [n]
  int32_t* parent;        // [max(n - 1, 1) + n]: internal nodes then leaves
  uint32_t* flags;        // [max(n - 1, 1)]: arrival counts of the bottom-up refit
  uint32_t* level_count;  // [kRefitLevels]: frontier size of each refit level
  uint32_t* hist;         // radix histogram scratch
  uint32_t* depth;        // [1]
  int32_t n;
  float lo[3], hi[3];
};
size_t radix_hist_words(int64_t n);
hipError_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                            uint32_t* hist, int64_t n, int key_bits, hipStream_t s, bool* result_in_alt);
hipError_t build_bvh(BvhBuild& b, hipStream_t s);
// Breadth-first copy of the 4-wide records reached from the root (src, nn
// records) into dst (nn records, the tail zero), children of a record in
// consecutive records; levels >= the tree's 4-wide depth.  front0 / front1:
// nn words each; lv: 2 kRelayoutLevels words.
constexpr int kRelayoutLevels = 128;
hipError_t relayout_wide(const float4* src, float4* dst, int64_t nn, uint32_t* front0, uint32_t* front1,
                         uint32_t* lv, int levels, hipStream_t s);

}  // namespace rtmc
