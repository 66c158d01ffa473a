// Linear BVH construction on the device.
//
// The paper tests every ray against every surface element and notes that this
// scan becomes prohibitive for large meshes (section 2.1).  The library
// replaces the scan with a binary BVH built in four device passes:
//   1. Morton code of each triangle centroid (21 bits per axis, 63 bits);
//   2. LSD radix sort of (code, triangle) pairs, 8 bits per pass;
//   3. the hierarchy of Karras (HPG 2012): internal node i covers the sorted
//      range decided by the longest common prefix of neighbouring codes, equal
//      codes being told apart by their indices;
//   4. bounds, bottom up, one launch per node height: a node is merged from
//      its two child boxes once the second child has arrived.
// Child boxes are stored in the parent (64-byte node record); k_collapse4
// then turns every binary node into the quantized 4-wide node traversal
// reads (up to four children per 64-byte record).
#include <algorithm>

#include "bvh_build.h"

namespace rtmc {

namespace {

constexpr int kSortBlock = 256;
constexpr int kSortWaves = kSortBlock / 64;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortBlock * kSortRounds;  // keys per workgroup

__device__ inline uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// ---------------------------------------------------------------- radix sort

__global__ __launch_bounds__(kSortBlock) void k_radix_hist(const uint64_t* __restrict__ keys, int64_t n,
                                                            int shift, uint32_t* __restrict__ hist,
                                                            int nblocks) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    int64_t k = base + (int64_t)r * kSortBlock + threadIdx.x;
    if (k < n) atomicAdd(&h[(uint32_t)(keys[k] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of len words by one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan_excl(uint32_t* __restrict__ a, int64_t len) {
  __shared__ uint32_t sums[1024];
  const int64_t per = (len + 1023) / 1024;
  const int64_t b = (int64_t)threadIdx.x * per;
  const int64_t e = b + per < len ? b + per : len;
  uint32_t s = 0;
  for (int64_t i = b; i < e; ++i) s += a[i];
  sums[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = threadIdx.x >= (unsigned)off ? sums[threadIdx.x - off] : 0u;
    __syncthreads();
    sums[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = threadIdx.x ? sums[threadIdx.x - 1] : 0u;
  for (int64_t i = b; i < e; ++i) {
    uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
}

// Exclusive scan of a long array in three launches: the sum of each 4096-word
// segment, an exclusive scan of those sums (k_scan_excl, one workgroup), then
// each segment scanned inside its workgroup and offset by its sum's prefix.
constexpr int kScanSeg = 4096;  // words per workgroup of 256 threads, 16 each

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* __restrict__ a, int64_t len,
                                                     uint32_t* __restrict__ part) {
  __shared__ uint32_t ws[4];
  const int64_t b0 = (int64_t)blockIdx.x * kScanSeg;
  uint32_t s = 0;
  for (int r = 0; r < 16; ++r) {
    const int64_t i = b0 + (int64_t)r * 256 + threadIdx.x;
    if (i < len) s += a[i];
  }
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ __launch_bounds__(256) void k_scan_apply(uint32_t* __restrict__ a, int64_t len,
                                                    const uint32_t* __restrict__ part) {
  __shared__ uint32_t ts[256];
  const int64_t b0 = (int64_t)blockIdx.x * kScanSeg + (int64_t)threadIdx.x * 16;
  uint32_t v[16], s = 0;
  for (int q = 0; q < 16; ++q) {
    v[q] = b0 + q < len ? a[b0 + q] : 0u;
    s += v[q];
  }
  ts[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t t = threadIdx.x >= (unsigned)off ? ts[threadIdx.x - off] : 0u;
    __syncthreads();
    ts[threadIdx.x] += t;
    __syncthreads();
  }
  uint32_t run = part[blockIdx.x] + ts[threadIdx.x] - s;
  for (int q = 0; q < 16; ++q) {
    if (b0 + q < len) a[b0 + q] = run;
    run += v[q];
  }
}

// Stable scatter: each wave owns kSortRounds * 64 consecutive keys of the
// tile; ranks inside a round come from ballots over the 8 digit bits.
__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(const uint64_t* __restrict__ kin,
                                                               const uint32_t* __restrict__ vin,
                                                               uint64_t* __restrict__ kout,
                                                               uint32_t* __restrict__ vout, int64_t n, int shift,
                                                               const uint32_t* __restrict__ hist, int nblocks) {
  __shared__ uint32_t goff[256];
  __shared__ uint32_t woff[kSortWaves][256];
  const int w = threadIdx.x / 64;
  const uint32_t lane = lane_id();
  goff[threadIdx.x] = hist[(size_t)threadIdx.x * nblocks + blockIdx.x];
  for (int i = 0; i < kSortWaves; ++i) woff[i][threadIdx.x] = 0;
  __syncthreads();
  const int64_t seg = (int64_t)blockIdx.x * kSortTile + (int64_t)w * (kSortRounds * 64);
  for (int r = 0; r < kSortRounds; ++r) {
    int64_t k = seg + r * 64 + lane;
    if (k < n) atomicAdd(&woff[w][(uint32_t)(kin[k] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  {
    const int d = threadIdx.x;
    uint32_t run = 0;
    for (int i = 0; i < kSortWaves; ++i) {
      uint32_t c = woff[i][d];
      woff[i][d] = run;
      run += c;
    }
  }
  __syncthreads();
  const uint64_t lt = (1ull << lane) - 1ull;
  for (int r = 0; r < kSortRounds; ++r) {
    int64_t k = seg + r * 64 + lane;
    bool valid = k < n;
    uint64_t key = valid ? kin[k] : 0ull;
    uint32_t val = valid ? vin[k] : 0u;
    uint32_t d = (uint32_t)(key >> shift) & 0xFFu;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      uint64_t m = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? m : ~m;
    }
    if (valid) {
      uint32_t rank = (uint32_t)__popcll(peers & lt);
      uint32_t pos = goff[d] + woff[w][d] + rank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    // the highest lane of each digit group advances that digit's offset
    if (valid && (peers >> lane) == 1ull) woff[w][d] += (uint32_t)__popcll(peers);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- Morton

__device__ inline uint64_t spread3(uint32_t v) {
  uint64_t x = 0;
  for (int i = 0; i < 21; ++i) x |= (uint64_t)((v >> i) & 1u) << (3 * i);
  return x;
}

__global__ void k_morton(const float4* __restrict__ tris, int32_t n, float lox, float loy, float loz, float sx,
                         float sy, float sz, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float4 a = tris[3 * (int64_t)i], b = tris[3 * (int64_t)i + 1], c = tris[3 * (int64_t)i + 2];
  float cx = (a.x + b.x + c.x) * (1.0f / 3.0f);
  float cy = (a.y + b.y + c.y) * (1.0f / 3.0f);
  float cz = (a.z + b.z + c.z) * (1.0f / 3.0f);
  const float q = 2097152.0f;  // 2^21
  uint32_t qx = (uint32_t)fminf(fmaxf((cx - lox) * sx * q, 0.0f), q - 1.0f);
  uint32_t qy = (uint32_t)fminf(fmaxf((cy - loy) * sy * q, 0.0f), q - 1.0f);
  uint32_t qz = (uint32_t)fminf(fmaxf((cz - loz) * sz * q, 0.0f), q - 1.0f);
  keys[i] = spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2);
  vals[i] = (uint32_t)i;
}

__global__ void k_gather_tris(const float4* __restrict__ in, const uint32_t* __restrict__ perm, int32_t n,
                              float4* __restrict__ out, float4* __restrict__ rot) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t s = 3 * (int64_t)perm[i];
  const float4 a = in[s], b = in[s + 1], c = in[s + 2];
  out[3 * (int64_t)i] = a;
  out[3 * (int64_t)i + 1] = b;
  out[3 * (int64_t)i + 2] = c;
  // the traversal record: x y z x y of each vertex, then a.w (caller's index)
  rot[4 * (int64_t)i] = make_float4(a.x, a.y, a.z, a.x);
  rot[4 * (int64_t)i + 1] = make_float4(a.y, b.x, b.y, b.z);
  rot[4 * (int64_t)i + 2] = make_float4(b.x, b.y, c.x, c.y);
  rot[4 * (int64_t)i + 3] = make_float4(c.z, c.x, c.y, a.w);
}

// ---------------------------------------------------------------- Karras

__device__ inline int prefix_len(const uint64_t* keys, int32_t n, int32_t i, int32_t j) {
  if (j < 0 || j >= n) return -1;
  uint64_t a = keys[i], b = keys[j];
  if (a == b) return 64 + __clz((uint32_t)(i ^ j));
  return __clzll(a ^ b);
}

__global__ void k_karras(const uint64_t* __restrict__ keys, int32_t n, float4* __restrict__ nodes,
                         int32_t* __restrict__ parent) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  const int d = prefix_len(keys, n, i, i + 1) - prefix_len(keys, n, i, i - 1) > 0 ? 1 : -1;
  const int dmin = prefix_len(keys, n, i, i - d);
  int32_t lmax = 2;
  while (prefix_len(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
  int32_t l = 0;
  for (int32_t t = lmax >> 1; t >= 1; t >>= 1)
    if (prefix_len(keys, n, i, i + (l + t) * d) > dmin) l += t;
  const int32_t j = i + l * d;
  const int dnode = prefix_len(keys, n, i, j);
  int32_t s = 0, step = l;
  do {
    step = (step + 1) >> 1;
    if (prefix_len(keys, n, i, i + (s + step) * d) > dnode) s += step;
  } while (step > 1);
  const int32_t g = i + s * d + (d < 0 ? -1 : 0);
  const int32_t lo = i < j ? i : j, hi = i < j ? j : i;
  uint32_t left, right;
  if (lo == g) {
    left = (uint32_t)g | kLeafBit;
    parent[(n - 1) + g] = i;
  } else {
    left = (uint32_t)g;
    parent[g] = i;
  }
  if (hi == g + 1) {
    right = (uint32_t)(g + 1) | kLeafBit;
    parent[(n - 1) + g + 1] = i;
  } else {
    right = (uint32_t)(g + 1);
    parent[g + 1] = i;
  }
  nodes[4 * (int64_t)i + 3] = make_float4(__uint_as_float(left), __uint_as_float(right), 0.0f, 0.0f);
  if (i == 0) parent[0] = -1;
}

__device__ inline void tri_box(const float4* tris, int32_t k, float b[6]) {
  float4 a = tris[3 * (int64_t)k], c = tris[3 * (int64_t)k + 1], e = tris[3 * (int64_t)k + 2];
  b[0] = fminf(fminf(a.x, c.x), e.x);
  b[1] = fminf(fminf(a.y, c.y), e.y);
  b[2] = fminf(fminf(a.z, c.z), e.z);
  b[3] = fmaxf(fmaxf(a.x, c.x), e.x);
  b[4] = fmaxf(fmaxf(a.y, c.y), e.y);
  b[5] = fmaxf(fmaxf(a.z, c.z), e.z);
}

__device__ inline void store_slot(float4* nodes, int32_t p, int slot, const float b[6]) {
  float* f = reinterpret_cast<float*>(nodes + 4 * (int64_t)p);
  const int o = slot * 6;
  for (int q = 0; q < 6; ++q) f[o + q] = b[q];
}

// Bottom-up bounds, one launch per node height.  Launch 0 writes every leaf's
// box into its slot of the parent record; launch L merges the two child boxes
// of every node whose taller child has height L - 1 (the frontier of level L),
// writes the union into the parent's slot and counts the arrival there.  The
// second child to arrive at a node appends it to the next level's frontier.
// A box is read only by a later launch than the one that wrote it, so the
// order of launches on the stream is all the synchronisation the boxes need;
// the arrival counts are relaxed atomic increments of one word each.  The
// launch that reaches the root records its level: the tree's depth in
// internal nodes (a leaf has height 0, a node one more than its taller child).
__device__ inline void arrive(float4* nodes, const int32_t* parent, uint32_t* flags, uint32_t child, int32_t p,
                              const float b[6], uint32_t* next, uint32_t* next_count) {
  const float4 links = nodes[4 * (int64_t)p + 3];
  store_slot(nodes, p, __float_as_uint(links.x) == child ? 0 : 1, b);
  if (atomicAdd(&flags[p], 1u) == 1u) next[atomicAdd(next_count, 1u)] = (uint32_t)p;
}

__global__ void k_refit_leaves(const float4* __restrict__ tris, int32_t n, float4* nodes,
                               const int32_t* __restrict__ parent, uint32_t* flags, uint32_t* next,
                               uint32_t* next_count) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  float b[6];
  tri_box(tris, k, b);
  arrive(nodes, parent, flags, (uint32_t)k | kLeafBit, parent[(n - 1) + k], b, next, next_count);
}

__global__ void k_refit_level(float4* nodes, const int32_t* __restrict__ parent, uint32_t* flags,
                              const uint32_t* __restrict__ front, const uint32_t* count, uint32_t* next,
                              uint32_t* next_count, uint32_t level, uint32_t* depth) {
  const uint32_t m = *count;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const int32_t p = (int32_t)front[i];
    const float4* r = nodes + 4 * (int64_t)p;
    const float4 r0 = r[0], r1 = r[1], r2 = r[2];  // slot 0: r0.xyzw r1.xy; slot 1: r1.zw r2.xyzw
    const float b[6] = {fminf(r0.x, r1.z), fminf(r0.y, r1.w), fminf(r0.z, r2.x),
                        fmaxf(r0.w, r2.y), fmaxf(r1.x, r2.z), fmaxf(r1.y, r2.w)};
    const int32_t q = parent[p];
    if (q < 0)
      *depth = level;
    else
      arrive(nodes, parent, flags, (uint32_t)p, q, b, next, next_count);
  }
}

// One triangle: a single node whose two children are that triangle.
__global__ void k_single(const float4* __restrict__ tris, float4* nodes) {
  float b[6];
  tri_box(tris, 0, b);
  store_slot(nodes, 0, 0, b);
  store_slot(nodes, 0, 1, b);
  nodes[3] = make_float4(__uint_as_float(kLeafBit), __uint_as_float(kLeafBit), 0.0f, 0.0f);
}

}  // namespace

size_t radix_hist_words(int64_t n) {
  int64_t nb = (n + kSortTile - 1) / kSortTile;
  if (nb < 1) nb = 1;
  const int64_t len = nb * 256;
  return (size_t)(len + (len + kScanSeg - 1) / kScanSeg + 16);  // histogram, then the segment sums
}

hipError_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt, uint32_t* hist,
                            int64_t n, int key_bits, hipStream_t s, bool* result_in_alt) {
  *result_in_alt = false;
  if (n <= 1) return hipSuccess;
  const int nb = (int)((n + kSortTile - 1) / kSortTile);
  uint64_t* ka = keys;
  uint32_t* va = vals;
  uint64_t* kb = keys_alt;
  uint32_t* vb = vals_alt;
  for (int shift = 0; shift < key_bits; shift += 8) {
    k_radix_hist<<<nb, kSortBlock, 0, s>>>(ka, n, shift, hist, nb);
    {
      const int64_t len = (int64_t)nb * 256;
      const int g = (int)((len + kScanSeg - 1) / kScanSeg);
      uint32_t* part = hist + len;
      k_scan_reduce<<<g, 256, 0, s>>>(hist, len, part);
      k_scan_excl<<<1, 1024, 0, s>>>(part, g);
      k_scan_apply<<<g, 256, 0, s>>>(hist, len, part);
    }
    k_radix_scatter<<<nb, kSortBlock, 0, s>>>(ka, va, kb, vb, n, shift, hist, nb);
    uint64_t* tk = ka;
    ka = kb;
    kb = tk;
    uint32_t* tv = va;
    va = vb;
    vb = tv;
    *result_in_alt = !*result_in_alt;
  }
  return hipGetLastError();
}

// 4-wide node of binary internal node i: i's two children, then, while fewer
// than four slots are filled, the inner slot of largest surface area replaced
// by its own two children (leaves stay as they are), so 2 to 4 slots.  Every
// binary node gets its 4-wide node (one thread per node), so a slot may link
// to a node of any depth; traversal reaches only the ones it links to.
//
// A node is 64 bytes (four float4): the origin o of the union box in words
// 0-2 and the three per-axis power-of-two scales s as floats in words 3, 14
// and 15; the four child links in words 4-7 (kEmpty: unused slot); the child
// boxes quantized to bytes, lo_x[4] lo_y[4] lo_z[4] hi_x[4] in words 8-11
// and hi_y[4] hi_z[4] in words 12-13.  A child's box decodes as fmaf(q, s, o) per bound, and the
// builder moves each code outwards until that decoded box contains the exact
// one; traversal's slab distances to the decoded planes carry a margin that
// covers their own rounding, so traversal stays conservative.
__device__ inline void load_node(const float4* nodes, int64_t i, float b0[6], float b1[6], uint32_t& l0,
                                 uint32_t& l1) {
  const float4 n0 = nodes[4 * i], n1 = nodes[4 * i + 1], n2 = nodes[4 * i + 2], n3 = nodes[4 * i + 3];
  b0[0] = n0.x;
  b0[1] = n0.y;
  b0[2] = n0.z;
  b0[3] = n0.w;
  b0[4] = n1.x;
  b0[5] = n1.y;
  b1[0] = n1.z;
  b1[1] = n1.w;
  b1[2] = n2.x;
  b1[3] = n2.y;
  b1[4] = n2.z;
  b1[5] = n2.w;
  l0 = __float_as_uint(n3.x);
  l1 = __float_as_uint(n3.y);
}

__device__ inline float pow2f(int e) { return __uint_as_float((uint32_t)(e + 127) << 23); }

// Power-of-two scale for an axis of extent w (>= 0): 255 steps cover w.
__device__ inline int axis_exp(float o, float hi) {
  const float w = fmaxf(hi - o, 1e-30f);
  int e;
  frexpf(w / 255.0f, &e);  // w / 255 < 2^e
  e = max(-126, min(127, e));
  while (e < 127 && fmaf(255.0f, pow2f(e), o) < hi) ++e;
  return e;
}

__device__ inline uint32_t q_lo(float v, float o, float sc) {
  int q = (int)floorf((v - o) / sc);
  q = max(0, min(255, q));
  while (q > 0 && fmaf((float)q, sc, o) > v) --q;
  return (uint32_t)q;
}

__device__ inline uint32_t q_hi(float v, float o, float sc) {
  int q = (int)ceilf((v - o) / sc);
  q = max(0, min(255, q));
  while (q < 255 && fmaf((float)q, sc, o) < v) ++q;
  return (uint32_t)q;
}

__global__ void k_collapse4(const float4* __restrict__ nodes, int64_t nn, float4* __restrict__ nodes4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  float b[4][6];
  uint32_t c[4];
  int k = 0;
  float cb[2][6];
  uint32_t cl[2];
  load_node(nodes, i, cb[0], cb[1], cl[0], cl[1]);
  for (int side = 0; side < 2; ++side) {
    for (int q = 0; q < 6; ++q) b[k][q] = cb[side][q];
    c[k++] = cl[side];
  }
  // greedy: expand the inner slot of largest surface area until four slots
  while (k < 4) {
    int best = -1;
    float ba = -1.0f;
    for (int j = 0; j < k; ++j) {
      if (c[j] & kLeafBit) continue;
      const float dx = b[j][3] - b[j][0], dy = b[j][4] - b[j][1], dz = b[j][5] - b[j][2];
      // unfused, so the choice is reproducible on the host
      const float area = __fadd_rn(__fadd_rn(__fmul_rn(dx, dy), __fmul_rn(dy, dz)), __fmul_rn(dz, dx));
      if (area > ba) {
        ba = area;
        best = j;
      }
    }
    if (best < 0) break;
    float g0[6], g1[6];
    uint32_t m0, m1;
    load_node(nodes, c[best], g0, g1, m0, m1);
    for (int q = 0; q < 6; ++q) b[best][q] = g0[q];
    c[best] = m0;
    for (int q = 0; q < 6; ++q) b[k][q] = g1[q];
    c[k++] = m1;
  }
  const int used = k;
  for (; k < 4; ++k) c[k] = kEmpty;
  float o[3], sc[3];
  int e[3];
  for (int a = 0; a < 3; ++a) {
    float lo = b[0][a], hi = b[0][3 + a];
    for (int j = 1; j < used; ++j) {
      lo = fminf(lo, b[j][a]);
      hi = fmaxf(hi, b[j][3 + a]);
    }
    o[a] = lo;
    e[a] = axis_exp(lo, hi);
    sc[a] = pow2f(e[a]);
  }
  uint32_t ql[3] = {0u, 0u, 0u}, qh[3] = {0u, 0u, 0u};
  for (int j = 0; j < used; ++j)
    for (int a = 0; a < 3; ++a) {
      ql[a] |= q_lo(b[j][a], o[a], sc[a]) << (8 * j);
      qh[a] |= q_hi(b[j][3 + a], o[a], sc[a]) << (8 * j);
    }
  float4* out = nodes4 + 4 * i;
  // the scales 2^e themselves (x in word 3, y and z in words 14 and 15), so
  // that traversal takes a plane's step as one product
  out[0] = make_float4(o[0], o[1], o[2], sc[0]);
  out[1] = make_float4(__uint_as_float(c[0]), __uint_as_float(c[1]), __uint_as_float(c[2]), __uint_as_float(c[3]));
  out[2] = make_float4(__uint_as_float(ql[0]), __uint_as_float(ql[1]), __uint_as_float(ql[2]), __uint_as_float(qh[0]));
  out[3] = make_float4(__uint_as_float(qh[1]), __uint_as_float(qh[2]), sc[1], sc[2]);
}

// ---------------------------------------------------------------- relayout

// One level of the breadth-first relayout of the 4-wide records.  Only the
// records reached from the root are kept (about half: the others belong to
// binary nodes absorbed into a parent's four slots), level after level, and
// the inner children of a record take consecutive records, so a line holds
// records that one ray visits together.  lv[0..kLevels) counts the records
// of each level, lv[kLevels + l] is the first record of level l; front_in
// lists the level's records by their index in the collapsed array.  A block
// takes one atomic for its threads' children (a scan in LDS); the order of
// blocks within a level, hence of records within it, is not fixed.
constexpr int kRelayoutBlock = 256;
typedef float f4v __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kRelayoutBlock) void k_relayout_level(const float4* __restrict__ src,
                                                                  float4* __restrict__ dst,
                                                                  const uint32_t* __restrict__ front_in,
                                                                  uint32_t* __restrict__ front_out,
                                                                  uint32_t* __restrict__ lv, int level) {
  __shared__ uint32_t s_cnt[kRelayoutBlock];
  __shared__ uint32_t s_base;
  const uint32_t n_in = lv[level];
  const uint32_t first = lv[kRelayoutLevels + level];
  const uint32_t next_first = first + n_in;
  if (blockIdx.x == 0 && threadIdx.x == 0) lv[kRelayoutLevels + level + 1] = next_first;
  for (uint32_t i0 = blockIdx.x * kRelayoutBlock; i0 < n_in; i0 += gridDim.x * kRelayoutBlock) {
    const uint32_t i = i0 + threadIdx.x;
    f4v r0 = {0, 0, 0, 0}, r1 = r0, r2 = r0, r3 = r0;
    uint32_t k = 0;
    if (i < n_in) {
      const float4* R = src + 4 * (size_t)front_in[i];
      r0 = *(const f4v*)&R[0];
      r1 = *(const f4v*)&R[1];
      r2 = *(const f4v*)&R[2];
      r3 = *(const f4v*)&R[3];
      for (int j = 0; j < 4; ++j) {
        const uint32_t l = __float_as_uint(r1[j]);
        k += (l != kEmpty && !(l & kLeafBit)) ? 1u : 0u;
      }
    }
    // exclusive scan of the block's child counts
    s_cnt[threadIdx.x] = k;
    __syncthreads();
    for (int off = 1; off < kRelayoutBlock; off <<= 1) {
      const uint32_t v = threadIdx.x >= (unsigned)off ? s_cnt[threadIdx.x - off] : 0u;
      __syncthreads();
      s_cnt[threadIdx.x] += v;
      __syncthreads();
    }
    const uint32_t incl = s_cnt[threadIdx.x];
    if (threadIdx.x == kRelayoutBlock - 1) s_base = atomicAdd(&lv[level + 1], incl);
    __syncthreads();
    uint32_t pos = s_base + incl - k;
    if (i < n_in) {
      for (int j = 0; j < 4; ++j) {
        const uint32_t l = __float_as_uint(r1[j]);
        if (l != kEmpty && !(l & kLeafBit)) {
          front_out[pos] = l;
          r1[j] = __uint_as_float(next_first + pos);
          ++pos;
        }
      }
      f4v* D = (f4v*)(dst + 4 * (size_t)(first + i));
      D[0] = r0;
      D[1] = r1;
      D[2] = r2;
      D[3] = r3;
    }
    __syncthreads();
  }
}

hipError_t relayout_wide(const float4* src, float4* dst, int64_t nn, uint32_t* front0, uint32_t* front1,
                         uint32_t* lv, int levels, hipStream_t s) {
  if (levels + 1 > kRelayoutLevels) return hipErrorInvalidValue;
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(dst), 0u, (size_t)nn * 16, s);
  if (e == hipSuccess) e = launch_fill_u32(lv, 0u, 2 * kRelayoutLevels, s);
  if (e == hipSuccess) e = launch_fill_u32(lv, 1u, 1, s);        // level 0: the root record
  if (e == hipSuccess) e = launch_fill_u32(front0, 0u, 1, s);    // ... which is record 0
  if (e != hipSuccess) return e;
  const int grid = (int)std::min<int64_t>((nn + kRelayoutBlock - 1) / kRelayoutBlock, 2048);
  for (int l = 0; l < levels; ++l) {
    k_relayout_level<<<grid, kRelayoutBlock, 0, s>>>(src, dst, (l & 1) ? front1 : front0, (l & 1) ? front0 : front1,
                                                     lv, l);
  }
  return hipGetLastError();
}

hipError_t build_bvh(BvhBuild& b, hipStream_t s) {
  const int32_t n = b.n;
  if (n <= 0) return hipSuccess;
  const int TB = 256;
  const int g = (n + TB - 1) / TB;
  float sx = 1.0f / (b.hi[0] - b.lo[0]), sy = 1.0f / (b.hi[1] - b.lo[1]), sz = 1.0f / (b.hi[2] - b.lo[2]);
  k_morton<<<g, TB, 0, s>>>(b.tris_in, n, b.lo[0], b.lo[1], b.lo[2], sx, sy, sz, b.keys, b.vals);
  bool alt = false;
  hipError_t e = radix_sort_pairs(b.keys, b.vals, b.keys_alt, b.vals_alt, b.hist, n, 63, s, &alt);
  if (e != hipSuccess) return e;
  uint64_t* keys = alt ? b.keys_alt : b.keys;
  uint32_t* perm = alt ? b.vals_alt : b.vals;
  k_gather_tris<<<g, TB, 0, s>>>(b.tris_in, perm, n, b.tris_out, b.tris_rot);
  if (n == 1) {
    k_single<<<1, 1, 0, s>>>(b.tris_out, b.nodes);
    k_collapse4<<<1, 64, 0, s>>>(b.nodes, 1, b.nodes4);
    return hipGetLastError();
  }
  const int gi = (n - 1 + TB - 1) / TB;
  k_karras<<<gi, TB, 0, s>>>(keys, n, b.nodes, b.parent);
  e = launch_fill_u32(b.flags, 0u, (size_t)(n - 1), s);  // arrival counts
  if (e == hipSuccess) e = launch_fill_u32(b.depth, 0u, 1, s);
  if (e == hipSuccess) e = launch_fill_u32(b.level_count, 0u, kRefitLevels, s);
  if (e != hipSuccess) return e;
  // frontiers of even and odd levels: two n-word halves of the key buffer,
  // free once the hierarchy is built
  uint32_t* front[2] = {reinterpret_cast<uint32_t*>(b.keys), reinterpret_cast<uint32_t*>(b.keys) + n};
  k_refit_leaves<<<g, TB, 0, s>>>(b.tris_out, n, b.nodes, b.parent, b.flags, front[1], b.level_count + 1);
  // the frontier sizes are only known on the device: launch a batch of levels,
  // then read whether the next level is empty
  const int grid = std::min(gi, 1024);
  const int kBatch = 16;
  for (int level = 1;; level += kBatch) {
    for (int l = level; l < level + kBatch; ++l) {
      if (l + 1 >= kRefitLevels) return hipErrorInvalidValue;  // deeper than any tree of distinct 63-bit keys
      k_refit_level<<<grid, TB, 0, s>>>(b.nodes, b.parent, b.flags, front[l & 1], b.level_count + l,
                                        front[(l + 1) & 1], b.level_count + l + 1, (uint32_t)l, b.depth);
    }
    uint32_t left = 0;
    e = hipMemcpyAsync(&left, b.level_count + level + kBatch, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (left == 0) break;
  }
  k_collapse4<<<gi, TB, 0, s>>>(b.nodes, (int64_t)(n - 1), b.nodes4);
  return hipGetLastError();
}

}  // namespace rtmc
