// Barnes-Hut interaction lists on the device: the lists of every bucket's work request, from a tree
// whose nodes are numbered in pre-order (children in ascending index, each node's ids contiguous).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gc {

struct WalkArgs {
  const int2* range;          // per node (first id, count)
  const double* com;          // per node centre of mass, 3 doubles
  const double* side;         // per node cube side
  const int32_t* skip;        // per node: index just past its subtree
  const float4* rec;          // per id (x, y, z, m)
  const int32_t* bucket_node; // per bucket: its leaf node
  int32_t n_nodes, n_buckets, n_ids;
  double theta;
  int32_t* n_first;           // count pass: per-bucket node count; fill pass: offsets (n_buckets + 1)
  int32_t* r_first;           // the same for direct ranges
  int32_t* node_idx;          // fill pass outputs
  int32_t* ranges;            // (first, count) pairs
  unsigned long long* bad;    // count of buckets whose leaf index or id range is invalid
  int32_t* sn;                // count pass: each bucket's first kWalkCapNodes node entries (or nullptr)
  int2* sr;                   // and first kWalkCapRanges ranges
};
// Per-bucket room of the count pass's copy of the lists; a bucket with more is walked again.
constexpr int kWalkCapNodes = 2048;
constexpr int kWalkCapRanges = 128;
// The walk without allocation: its scratch (256 bytes of totals, then 4 bytes per node) is a fixed
// device array of 8 MiB + 256 bytes, so trees of up to 2^21 nodes.
constexpr int kWalkNoAllocMaxNodes = 1 << 21;
constexpr size_t kWalkScratchBytes = 256 + sizeof(int32_t) * (size_t)kWalkNoAllocMaxNodes;

hipError_t launch_subtree_end(const int2* range, int32_t n_nodes, int32_t* skip, hipStream_t s);
hipError_t launch_walk(bool fill, const WalkArgs& a, hipStream_t s);
// After the scan: the lists of every bucket that fit the count pass's room, copied to their offsets.
hipError_t launch_walk_copy(const WalkArgs& a, hipStream_t s);
// In-place exclusive scan of two count arrays of n entries (entry n receives the total); the two
// totals, as 64-bit sums, go to totals[0] and totals[1].
hipError_t launch_scan_counts(int32_t* a, int32_t* b, int32_t n, long long* totals, hipStream_t s);

}  // namespace gc
