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
constexpr int32_t kEmitPaper = 1;         // DevTables::emission of the paper's one/two-daughter rule
constexpr int kMaxGen = 10;
constexpr int kWrapMax = 10000;
constexpr float kSpawnEps = 1e-4f;
constexpr int kMaxEbins = 1024;
constexpr int kMaxAbins = 360;
constexpr int kMaxZbins = 256;
constexpr int kMaxYield = 8192;
constexpr int kMaxCdf = 1024;
constexpr int kGuide = 1024;  // entries of each CDF guide table
constexpr int kGlobalStack = 64;  // minimum traversal stack entries per lane beyond the LDS part
constexpr int kClaimMax = 2048;   // largest block of rays one traversal wave claims at once
constexpr int kShadeJobs = 32;    // chunks with at most this many jobs tally per workgroup in LDS

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

struct DevTables {
  const float* yld;
  const float* cdfE;
  const float* cdfF;
  const float* esee;  // E_SEE on the yield grid (paper emission), else null
  // guide tables of the CDF look-ups (kGuide entries each): gF[b] = first
  // segment whose upper CDF value reaches b / kGuide; gE[b] = last node at or
  // below the energy with bit pattern e1bits + (b << eshift), e1bits = cdfE[1]
  const uint16_t* gF;
  const uint16_t* gE;
  uint32_t e1bits, eshift;
  int32_t nE, nth, ncdf;
  int32_t emission;   // RTMC_EMIT_SPECTRUM or RTMC_EMIT_PAPER
  float logEmin, invdlogE, thscale, Ec;
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
  uint32_t* err;   // bit 1: stack overflow
};

struct ShadeArgs {
  const DevJob* jobs;
  int32_t n_jobs;
  DevTables tb;
  RayQueue qin, qout;
  uint32_t qcap;
  const uint32_t* count_in;
  uint32_t n_gen0;
  uint64_t chunk_lo;
  uint32_t* count_out;
  uint32_t* ppc;  // per-primary escape counts of the chunk
  int32_t gen, max_gen;
  int32_t n_ebins, n_abins, n_zbins;  // histogram bins: escaped energy, escape angle, absorption depth
  int32_t j_lo, j_hi;  // jobs overlapping the chunk
  HitRecs hit;
  uint32_t* err;  // bit 0: queue overflow
};

// host-side launchers (defined in the .hip files)
size_t traverse_lds_bytes(int lds_stack, int block);
// LDS of a shading workgroup; n_jobs = jobs of the chunk (tallied in LDS when <= kShadeJobs)
size_t shade_lds_bytes(const DevTables& tb, int n_hist, int block, int n_jobs);  // n_hist: all histogram bins
hipError_t launch_traverse(const TraverseArgs& a, bool multi, int occupancy, int grid, int block, hipStream_t s);
hipError_t launch_shade(const ShadeArgs& a, int n_cu, int block, hipStream_t s);  // grid = n_cu x occupancy
hipError_t launch_primaries(const DevJob* jobs, int32_t j_lo, int32_t j_hi, uint64_t chunk_lo, uint32_t n,
                            const RayQueue& q, hipStream_t s);
hipError_t launch_hit_ids(const float4* tris, const int32_t* code, int64_t n, int32_t* out, hipStream_t s);
hipError_t launch_chunk_reduce(const DevJob* jobs, int32_t j_lo, int32_t j_hi, const uint32_t* ppc, uint32_t n,
                               uint64_t chunk_lo, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, size_t n, hipStream_t s);
hipError_t launch_copy_probe(float4* dst, const float4* src, size_t n16, int grid, hipStream_t s);

// Surrogate MLP pieces (mlp.hip)
enum MlpEpi { MLP_EPI_F32 = 0, MLP_EPI_FWD_GELU = 1, MLP_EPI_BWD_GELU = 2 };

// C = A B^T, A [M, K] and B [N, K] bf16 row-major, K % 32 == 0, FP32 accumulation.
//   MLP_EPI_F32:      C[m, n] (float, ldc)
//   MLP_EPI_FWD_GELU: z = acc + bias[n]; Z[m, n] = z (if Z); H[m, n] = GELU(z) (bf16); Ht[n, m] likewise (if Ht)
//   MLP_EPI_BWD_GELU: d = acc * GELU'(Zs[m, n]); H[m, n] = d (bf16); Ht[n, m] likewise (if Ht)
struct MlpGemm {
  const __bf16* A;
  const __bf16* B;
  int M, N, K, lda, ldb;
  int epi;
  const float* bias;
  float* Z;
  int ldz;
  __bf16* H;
  int ldh;
  __bf16* Ht;
  int ldht;
  float* C;
  int ldc;
  const float* Zs;
};
hipError_t mlp_gemm(const MlpGemm& g, hipStream_t s);
hipError_t mlp_pack_input(const float* x, int B, int n_in, __bf16* X, __bf16* Xt, hipStream_t s);
hipError_t mlp_out_fwd(const __bf16* H, int B, int width, const float* w, const float* c, float* y, hipStream_t s);
hipError_t mlp_mse(const float* y, const float* t, int B, float* dy, float* acc, hipStream_t s);
hipError_t mlp_out_bwd_hidden(const float* dy, const float* w, const float* Z, int B, int width, __bf16* G,
                              __bf16* Gt, hipStream_t s);
hipError_t mlp_rowsum(const __bf16* Mt, int R, int B, const float* scale, float* out, hipStream_t s);
hipError_t mlp_adamw(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                     float wd, float c1, float c2, hipStream_t s);
hipError_t mlp_to_bf16(const float* W, int rows, int cols, __bf16* Wb, __bf16* Wtb, hipStream_t s);

// Fused inference of the 4 x 256 GELU network: y[r] = wout . H4(x[r]) + bout
// for r < n.  Hidden weights are the bf16 copies in [256, kin] layout
// (kin = 32 for layer 1, columns >= n_in zero); n_in <= 32.
struct MlpInfer {
  const float* x;  // [n, n_in]
  int64_t n;
  int n_in;
  const __bf16* W[4];
  const float* bias[4];
  const float* wout;  // [256]
  const float* bout;  // [1]
  float* y;           // [n]
};
hipError_t mlp_infer(const MlpInfer& p, hipStream_t s);

// BVH builder pieces
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
  uint32_t* flags;        // [2 max(n - 1, 1)]: arrival counts, then node heights
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
