// Internal structures shared by the library's HIP sources (not installed).
//
// Device data layout (all in HBM):
//   triangles  float4 [3 * n_tris], Morton order after the BVH build: V0, V1,
//              V2 of one triangle in 48 consecutive bytes; V0.w holds the
//              caller's triangle index (int32 bits).
//   rotated    float4 [4 * n_tris], what traversal reads: one 64-byte record
//   triangles  per sorted triangle, each vertex as five floats (x, y, z, x, y)
//              so that every cyclic order of its coordinates is three
//              consecutive floats, then the caller's triangle index.
//   BVH nodes  float4 [4 * n_nodes], binary: one 64-byte record per internal
//              node (both child boxes and both child links); kept for the
//              download and its structure tests.
//   4-wide     float4 [4 * n_nodes], what traversal reads: one 64-byte record
//              per binary node (union-box origin, three power-of-two scales,
//              four child links, the child boxes quantized to bytes), read
//              with four 16-byte loads from one cache line.
//   ray queue  structure of arrays, ten 32-bit streams, written and read
//              coalesced by whole waves.
//   hit records structure of arrays, seven 32-bit streams, one entry per ray
//              of the generation being processed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtmc {

constexpr uint32_t kLeafBit = 0x80000000u;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;  // unused child slot of a 4-wide node
constexpr int kMaxGen = 10;
constexpr int kWrapMax = 10000;
constexpr float kSpawnEps = 1e-4f;
constexpr int kMaxEbins = 1024;
constexpr int kMaxAbins = 360;
constexpr int kMaxZbins = 256;
constexpr int kMaxYield = 8192;
constexpr int kMaxCdf = 1024;
constexpr int kGlobalStack = 64;  // minimum traversal stack entries per lane beyond the LDS part
constexpr int kClaimDefault = 2048;  // largest block of rays one traversal wave claims at once (default)
constexpr int kClaimLimit = 8192;    // upper bound of that launch knob

// tally counter slots (u64 each), followed by the energy and angle histograms
enum TallySlot {
  T_RAYS = 0,
  T_ESCAPED,
  T_ABSORBED,
  T_TRUNCATED,
  T_LOST,
  T_SUBSTRATE,
  T_WRAPS,
  T_VISITS,
  T_TESTS,
  T_E_ESC_FX,  // escaped energy, 2^-20 eV fixed point
  T_E_DEP_FX,  // deposited energy, same units (two's complement sums)
  T_SPAWNED,
  T_C2,        // sum over primaries of (escape count)^2
  T_DROPPED,   // daughters that did not fit the queue
  T_STACKOVF,  // rays whose traversal stack overflowed
  T_SPARE,
  T_NCOUNT
};

constexpr double kFixScale = 1048576.0;  // 2^20

struct DevScene {
  const float4* nodes;  // quantized 4-wide nodes, 4 float4 each
  const float4* tris;    // sorted triangles, 48 B each
  const float4* tris_t;  // the same as rotated records, 64 B each (traversal)
  float lo[3], hi[3];
  float wext;  // bound on the magnitude of every coordinate of the scene and its node planes
  int32_t n_tris;
  uint32_t flags;
};

// One job: a scene traced at one (E, theta) point.
struct DevJob {
  DevScene sc;
  float E0;
  float theta;  // >= 0 fixed; < 0 uniform in [0, -theta]
  uint64_t seed;
  uint64_t pid0;   // primary id of the job's first primary
  uint64_t n_prim;
  uint64_t gbase;  // index of the job's first primary in the concatenated primary space
  unsigned long long* tally;
  uint32_t* pp_escaped;  // optional, indexed by primary id - pid0
};

struct RayQueue {
  float *ox, *oy, *oz, *dx, *dy, *dz, *E;
  uint32_t* path;
  uint32_t* ci;    // primary's index within the current chunk
  uint32_t* meta;  // gen (4 bits) | job << 4
};

// Per-ray result of the traversal launch (structure of arrays).
struct HitRecs {
  int32_t* code;  // sorted triangle index, or -1 escape, -2 substrate, -3 lost
  float* f0;      // barycentric weight of V1, or substrate x
  float* f1;      // barycentric weight of V2, or substrate y
  float* t;       // path length over all periodic segments
  uint32_t* visits;
  uint32_t* tests;
  uint32_t* wraps;  // bit 31: traversal stack overflowed
};

struct TraverseArgs {
  const DevJob* jobs;
  int32_t n_jobs;
  int32_t src;               // 1: queue, 2: explicit rays
  RayQueue qin;
  const float* rays;         // src 2: [n][6]
  uint32_t count;            // ray count when count_in is null
  const uint32_t* count_in;  // queue length in device memory, or null
  uint32_t qcap;
  uint64_t chunk_lo;
  HitRecs hit;
  uint32_t* work;
  uint32_t* gstack;
  int32_t lds_stack;
  int32_t gstack_depth;
  int32_t refill;  // refill a wave once this many lanes are idle
  uint32_t claim_max;  // largest block of rays a wave claims at once
  uint32_t* err;   // bit 1: stack overflow
};

// host-side launchers (traverse.hip; the fills and copies in shade.hip)
size_t traverse_lds_bytes(int lds_stack, int block);
hipError_t launch_traverse(const TraverseArgs& a, bool multi, int occupancy, int grid, int block, hipStream_t s);
hipError_t launch_primaries(const DevJob* jobs, int32_t j_lo, int32_t j_hi, uint64_t chunk_lo, uint32_t n,
                            const RayQueue& q, hipStream_t s);
hipError_t launch_hit_ids(const float4* tris, const int32_t* code, int64_t n, int32_t* out, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
// The first min(*count, qcap, n_max) rays of a queue as [n][6] (origin, direction); the number to *n_out.
hipError_t launch_copy_rays(const RayQueue& q, const uint32_t* count, uint32_t qcap, float* out, uint32_t n_max,
                            uint32_t* n_out, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, size_t n, hipStream_t s);
hipError_t launch_copy_probe(float4* dst, const float4* src, size_t n16, int grid, hipStream_t s);

}  // namespace rtmc
