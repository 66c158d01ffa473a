// Ray tracing Monte Carlo on gfx950: one lane per ray.
//
// A generation of rays (the paper's tree of branches, section 2.2, handled
// breadth-first across all primaries) is processed by two launches:
//   k_traverse: closest front-facing triangle by BVH traversal (section 2.1):
//     conservative slab tests against the four byte-quantized child boxes of
//     a 64-byte node and the watertight ray/triangle test of Woop, Benthin and
//     Wald (JCGT 2013) with back-face culling; periodic re-entry through the
//     x / y faces, escape through z_max, substrate plane at z_min (section
//     2.2).  Persistent waves whose lanes refill from the generation's queue
//     once enough of them are done.  Output: one 28-byte hit record per ray.
//   k_shade: the local incidence angle and the flat-surface tables give the
//     daughter count (stochastic rounding, footnote of section 2.2), energies
//     (inverse of the tabulated CDF truncated to the energy still available)
//     and cosine-law directions; daughters are appended to the next queue with
//     one atomic per workgroup step; tallies accumulate per lane and per job.
// Generation 0 is written to the queue from primary ids by k_primaries, so
// both launches read it like any other generation.  Random numbers:
// Philox4x32-10 (Salmon et al., SC'11) keyed by the job seed, counter (primary
// id, 0, path code, draw); draw 0 = birth of a primary, 1 = daughter count,
// 2 + d = daughter d; a daughter's path code is parent * 8 + d + 1.
#include "rtmc_internal.h"

namespace rtmc {
namespace {

// Explicit address spaces: pointers that arrive through the job table or the
// argument struct are otherwise generic, and generic (flat) accesses wait on
// both the vector-memory and the LDS counters.
#define GAS __attribute__((address_space(1)))
#define LAS __attribute__((address_space(3)))
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T>
__device__ inline GAS T* gp(T* p) {
  return (GAS T*)p;
}
template <typename T>
__device__ inline const GAS T* gp(const T* p) {
  return (const GAS T*)p;
}

constexpr float kPi = 3.14159265358979323846f;
constexpr float kDeg = 57.295779513082320876f;  // 180 / pi
// Absolute margin of the node slab distances, per unit of coordinate
// magnitude and of |1/d|: 1.05 * 2^-20 (see slab_margins).
constexpr float kSlack = 1.05f / 1048576.0f;

__device__ inline uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------- Philox

struct U4 {
  uint32_t x, y, z, w;
};

__device__ inline U4 philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

// (0, 1]: ((u >> 8) + 1) * 2^-24, exact in FP32
__device__ inline float u01(uint32_t u) { return (float)((u >> 8) + 1u) * 5.9604644775390625e-8f; }

// ---------------------------------------------------------------- geometry

// Per-lane ray state kept in registers while a segment is traversed (the
// direction itself is read only when a segment begins or ends, and waits in
// LDS meanwhile).
struct RayP {
  float ox, oy, oz;
  float ix, iy, iz;
  float w;  // slab margin of the current segment per unit of |1/d|
  float Sx, Sy, Sz;
  float qx, qy, qz;  // origin with its coordinates in the order kx, ky, kz
  uint32_t kk;       // 4 kx (byte offset of a rotated vertex) | bit 31 when kx and ky are swapped
};

__device__ inline float pick(float x, float y, float z, int k) { return k == 0 ? x : (k == 1 ? y : z); }

// Hardware reciprocal (1 ulp); tiny components are replaced so that slab
// distances stay finite and keep their sign.
__device__ inline float safe_inv(float d) {
  return __builtin_amdgcn_rcpf(fabsf(d) > 1e-20f ? d : copysignf(1e-20f, d));
}

__device__ inline void ray_setup(RayP& r, float dx, float dy, float dz) {
  r.ix = safe_inv(dx);
  r.iy = safe_inv(dy);
  r.iz = safe_inv(dz);
  const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
  // kz: the dominant axis; (kx, ky, kz) in cyclic order.  Written as selects
  // on the comparisons (an index into the three values would go to scratch).
  const bool z0 = ax > ay && ax > az, z1 = !z0 && ay > az;
  const float dkz = z0 ? dx : (z1 ? dy : dz);
  const float dkx = z0 ? dy : (z1 ? dz : dx);
  const float dky = z0 ? dz : (z1 ? dx : dy);
  // The watertight test keeps the sheared frame right-handed by swapping kx
  // and ky when d[kz] < 0.  The swap maps the edge functions U, V, W to
  // exactly -U, -V, -W (the same rounded products, subtracted the other way
  // round) and leaves T / det and the weights unchanged, so the test below
  // always uses the cyclic order and negates instead: the cyclic order is
  // what a rotated vertex record holds (kx = 1, 2, 0 for kz = 0, 1, 2).
  r.kk = (z0 ? 4u : (z1 ? 8u : 0u)) | (dkz < 0.0f ? 0x80000000u : 0u);
  // any per-ray shear is watertight as long as every triangle sees the same one
  r.Sz = __builtin_amdgcn_rcpf(dkz);
  r.Sx = dkx * r.Sz;
  r.Sy = dky * r.Sz;
}

// Origin in the shear's axis order (after every change of the origin).
__device__ inline void rotate_origin(RayP& r) {
  const bool x1 = (r.kk & 0xFu) == 4u, x2 = (r.kk & 0xFu) == 8u;
  r.qx = x1 ? r.oy : (x2 ? r.oz : r.ox);
  r.qy = x1 ? r.oz : (x2 ? r.ox : r.oy);
  r.qz = x1 ? r.ox : (x2 ? r.oy : r.oz);
}

// Margins of the fused slab distances of one segment.  A node's child plane
// is at b = fma(q, s, o) (s a power of two, so q*s*ix is exact); its distance
// is taken as fma(q, s*ix, (o - O)*ix -/+ m) in place of (b - O)*ix.  With
// every coordinate (planes, node origins, ray origin) bounded by W in
// magnitude, the rounding of b, of o - O and of the two fused operations
// moves that distance by at most about 5 * 2^-24 * W * |ix|, and the
// relative error of the reciprocal and the last rounding (3 ulp of a
// distance of at most 2 W |ix|) by at most 6 * 2^-24 * W * |ix|.  The
// margin m = 16.8 * 2^-24 * W * |ix| exceeds both together, so the near
// distance never exceeds the exact one and the far distance never falls
// short of it: the slab test is conservative without a relative factor.
// W takes the scene's coordinate bound (which covers decoded planes and
// node origins) and the segment origin, so rays from outside the cell are
// covered too.
__device__ inline void slab_margins(RayP& r, float wext) {
  r.w = fmaxf(fmaxf(wext, fabsf(r.ox)), fmaxf(fabsf(r.oy), fabsf(r.oz))) * kSlack;
}

// Slab test of one child from its near and far distances per axis.
__device__ inline bool box_hit(float nx, float ny, float nz, float fx, float fy, float fz, float tmax, float& tn) {
  const float t0 = fmaxf(fmaxf(nx, ny), fmaxf(nz, 0.0f));
  const float t1 = fminf(fminf(fx, fy), fz);
  tn = t0;
  return t0 <= fminf(t1, tmax);
}

// Watertight ray/triangle test with back-face culling.  a, b, c are the
// vertices with their coordinates already in the order kx, ky, kz (read from
// the rotated records); U, V, W are the sheared edge functions (weights of
// V0, V1, V2), negated when the ray's frame swaps kx and ky.  Products are
// kept unfused so that an edge shared by two triangles gets exactly opposite
// values, and an exactly zero edge function is recomputed in FP64.
__device__ inline bool tri_test(const RayP& r, float3 a, float3 b, float3 c, float tbest, float& t, float& b1,
                                float& b2) {
  const float ax = a.x - r.qx, ay = a.y - r.qy, Akz = a.z - r.qz;
  const float bx = b.x - r.qx, by = b.y - r.qy, Bkz = b.z - r.qz;
  const float cx = c.x - r.qx, cy = c.y - r.qy, Ckz = c.z - r.qz;
  const float Ax = fmaf(-r.Sx, Akz, ax), Ay = fmaf(-r.Sy, Akz, ay);
  const float Bx = fmaf(-r.Sx, Bkz, bx), By = fmaf(-r.Sy, Bkz, by);
  const float Cx = fmaf(-r.Sx, Ckz, cx), Cy = fmaf(-r.Sy, Ckz, cy);
  float U = __fsub_rn(__fmul_rn(Cx, By), __fmul_rn(Cy, Bx));
  float V = __fsub_rn(__fmul_rn(Ax, Cy), __fmul_rn(Ay, Cx));
  float W = __fsub_rn(__fmul_rn(Bx, Ay), __fmul_rn(By, Ax));
  if (U == 0.0f || V == 0.0f || W == 0.0f) {
    U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
    V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
    W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
  }
  const uint32_t sg = r.kk & 0x80000000u;
  U = __uint_as_float(__float_as_uint(U) ^ sg);
  V = __uint_as_float(__float_as_uint(V) ^ sg);
  W = __uint_as_float(__float_as_uint(W) ^ sg);
  if (U < 0.0f || V < 0.0f || W < 0.0f) return false;
  const float det = U + V + W;
  if (!(det > 0.0f)) return false;
  const float T = U * (r.Sz * Akz) + V * (r.Sz * Bkz) + W * (r.Sz * Ckz);
  if (!(T > 0.0f) || T > tbest * det) return false;
  const float inv = 1.0f / det;
  t = T * inv;
  b1 = V * inv;
  b2 = W * inv;
  return true;
}

// ---------------------------------------------------------------- tables (LDS)

// Value of a table on the yield grid at (E, alpha): bilinear in (ln E, alpha),
// clamped at the edges (the yield from LDS, E_SEE from global memory).
template <typename P>
__device__ inline float table_yield(P yld, const DevTables& tb, float E, float alpha) {
  float x = (logf(E) - tb.logEmin) * tb.invdlogE;
  x = fminf(fmaxf(x, 0.0f), (float)(tb.nE - 1));
  int i = min((int)floorf(x), tb.nE - 2);
  const float fx = x - (float)i;
  float y = fminf(fmaxf(alpha * tb.thscale, 0.0f), (float)(tb.nth - 1));
  int j = min((int)floorf(y), tb.nth - 2);
  const float fy = y - (float)j;
  const P row0 = yld + i * tb.nth + j;
  const P row1 = row0 + tb.nth;
  return (1.0f - fx) * (1.0f - fy) * row0[0] + fx * (1.0f - fy) * row1[0] + (1.0f - fx) * fy * row0[1] +
         fx * fy * row1[1];
}

// Piecewise-linear CDF at E.  The segment (last node at or below E) starts
// from a guide table over the bit patterns of positive energies, which are
// ordered like the energies, and moves forward; it is the segment a binary
// search would find.
__device__ inline float cdf_at(const LAS float* cE, const LAS float* cF, int n, const LAS uint16_t* gE,
                               uint32_t e1bits, uint32_t eshift, float E) {
  if (E <= cE[0]) return cF[0];
  if (E >= cE[n - 1]) return cF[n - 1];
  int lo = 0;
  if (E >= cE[1]) {
    const uint32_t b = (__float_as_uint(E) - e1bits) >> eshift;
    lo = gE[b < (uint32_t)kGuide ? b : (uint32_t)kGuide - 1u];
    while (cE[lo + 1] <= E) ++lo;
  }
  return cF[lo] + (E - cE[lo]) / (cE[lo + 1] - cE[lo]) * (cF[lo + 1] - cF[lo]);
}

// Energy where the piecewise-linear CDF first reaches c (0 < c <= 1): the
// first node m >= 1 with cF[m] >= c, starting from the guide table's lower
// bound for c.
__device__ inline float cdf_inv(const LAS float* cE, const LAS float* cF, int n, const LAS uint16_t* gF, float c) {
  if (!(cF[n - 1] >= c)) return cE[n - 1];
  const int b = min(max((int)(c * (float)kGuide), 0), kGuide - 1);
  int k = gF[b];
  while (!(cF[k + 1] >= c)) ++k;
  const float f0 = cF[k], f1 = cF[k + 1];
  if (f1 <= f0) return cE[k];
  return cE[k] + (c - f0) / (f1 - f0) * (cE[k + 1] - cE[k]);
}

// Orthonormal frame completing unit n (Duff et al., JCGT 2017).
__device__ inline void onb(float nx, float ny, float nz, float3& t1, float3& t2) {
  const float sign = copysignf(1.0f, nz);
  const float a = -1.0f / (sign + nz);
  const float b = nx * ny * a;
  t1 = make_float3(1.0f + sign * nx * nx * a, sign * b, -sign * nx);
  t2 = make_float3(b, sign + ny * ny * a, -ny);
}

// Job of concatenated primary index g among jobs [lo, hi] (sorted by gbase).
__device__ inline int find_job(const DevJob* jobs, int lo, int hi, uint64_t g) {
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (gp(jobs)[mid].gbase <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ inline long long to_fx(float E) { return (long long)llrintf(E * 1048576.0f); }

// ---------------------------------------------------------------- tallies

// Per-wave tallies.  Event counters and sums live in per-lane registers and
// are reduced across the wave only when the wave flushes; the two histograms
// are per-wave LDS blocks (their bins are spread, so LDS atomics rarely
// collide).
struct WaveTally {
  uint32_t c[T_NCOUNT];  // counter slots except the two energy sums
  unsigned long long e_esc, e_dep;
  LAS uint32_t* eh;  // LDS [n_ebins]
  LAS uint32_t* ah;  // LDS [n_abins]
  LAS uint32_t* zh;  // LDS [n_zbins]
};

__device__ inline void gadd(unsigned long long* g, unsigned long long v) {
  __hip_atomic_fetch_add(gp(g), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ inline void ladd(LAS T* p, T v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Workgroup-wide LDS tally blocks, one per job of the chunk (when few enough):
// [T_NCOUNT u64 counters][n_ebins u32][n_abins u32][n_zbins u32] per job.
struct JobTab {
  LAS unsigned char* base;
  int stride, n_eb, n_ab, j_lo, J;
};

__device__ inline LAS unsigned long long* jt_cnt(const JobTab& t, int job) {
  return (LAS unsigned long long*)(t.base + (size_t)(job - t.j_lo) * t.stride);
}
__device__ inline LAS uint32_t* jt_eh(const JobTab& t, int job) {
  return (LAS uint32_t*)(t.base + (size_t)(job - t.j_lo) * t.stride + T_NCOUNT * 8);
}

// slot is a compile-time constant at every call site.  A lane whose ray belongs
// to another job than its wave's tally adds directly: to that job's LDS block
// when the workgroup keeps one per job (jt), else to global memory.
__device__ inline void tally_cnt(bool mine, WaveTally& wt, unsigned long long* g, int slot, unsigned long long v,
                                 const JobTab* jt, int job) {
  if (!mine) {
    if (jt)
      ladd(jt_cnt(*jt, job) + slot, v);
    else
      gadd(g + slot, v);
  } else if (slot == T_E_ESC_FX) {
    wt.e_esc += v;
  } else if (slot == T_E_DEP_FX) {
    wt.e_dep += v;
  } else {
    wt.c[slot] += (uint32_t)v;
  }
}

__device__ inline unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline void flush_wave_lds(WaveTally& wt, LAS unsigned long long* cnt, uint32_t lane) {
#pragma unroll
  for (int k = 0; k < T_NCOUNT; ++k) {
    if (k == T_E_ESC_FX || k == T_E_DEP_FX || k == T_C2 || k == T_SPARE) continue;
    const unsigned long long v = wave_sum((unsigned long long)wt.c[k]);
    if (lane == 0 && v) ladd(cnt + k, v);
    wt.c[k] = 0u;
  }
  const unsigned long long ee = wave_sum(wt.e_esc), ed = wave_sum(wt.e_dep);
  if (lane == 0) {
    if (ee) ladd(cnt + T_E_ESC_FX, ee);
    if (ed) ladd(cnt + T_E_DEP_FX, ed);
  }
  wt.e_esc = 0ull;
  wt.e_dep = 0ull;
}

__device__ inline void flush_wave(WaveTally& wt, unsigned long long* g, int n_eb, int n_ab, int n_zb, uint32_t lane) {
#pragma unroll
  for (int k = 0; k < T_NCOUNT; ++k) {
    if (k == T_E_ESC_FX || k == T_E_DEP_FX || k == T_C2 || k == T_SPARE) continue;
    const unsigned long long v = wave_sum((unsigned long long)wt.c[k]);
    if (lane == 0 && v) gadd(g + k, v);
    wt.c[k] = 0u;
  }
  const unsigned long long ee = wave_sum(wt.e_esc), ed = wave_sum(wt.e_dep);
  if (lane == 0) {
    if (ee) gadd(g + T_E_ESC_FX, ee);
    if (ed) gadd(g + T_E_DEP_FX, ed);
  }
  wt.e_esc = 0ull;
  wt.e_dep = 0ull;
  wave_sync();
  for (int i = lane; i < n_eb; i += 64) {
    const uint32_t v = wt.eh[i];
    if (v) gadd(g + T_NCOUNT + i, (unsigned long long)v);
    wt.eh[i] = 0u;
  }
  for (int i = lane; i < n_ab; i += 64) {
    const uint32_t v = wt.ah[i];
    if (v) gadd(g + T_NCOUNT + n_eb + i, (unsigned long long)v);
    wt.ah[i] = 0u;
  }
  for (int i = lane; i < n_zb; i += 64) {
    const uint32_t v = wt.zh[i];
    if (v) gadd(g + T_NCOUNT + n_eb + n_ab + i, (unsigned long long)v);
    wt.zh[i] = 0u;
  }
  wave_sync();
}

__device__ inline uint32_t wave_incl_scan(uint32_t v, uint32_t lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(v, off, 64);
    if (lane >= (uint32_t)off) v += o;
  }
  return v;
}

// ---------------------------------------------------------------- traversal

enum { K_HIT = 0, K_ESCAPE = 1, K_SUBSTRATE = 2, K_LOST = 3 };

// Scene fields one lane needs while it traverses.
struct LaneScene {
  const float4* nodes;
  const float4* tris;
  int32_t n_tris;
  uint32_t flags;
};

// Per-lane traversal state: the current periodic segment of one ray.
struct Trav {
  RayP r;
  float t;        // closest hit so far (starts at the segment's exit distance)
  float b1, b2;   // barycentric weights of V1, V2 at the hit
  int32_t idx;    // sorted triangle index of the hit, -1 none
  int32_t oid;    // caller's triangle index of the hit
  uint32_t node;
  int sp;
  float total;  // path length of earlier segments
  int wraps;
};

// Distances from the segment origin to the x, y, z faces of the cell, with
// the ray's reciprocal direction (recomputed where needed, not kept live).
__device__ inline void exit_dists(const RayP& r, float dx, float dy, float dz, const DevScene& sc, float& te0,
                                  float& te1, float& te2) {
  const float tex = dx > 0.0f ? (sc.hi[0] - r.ox) * r.ix : (dx < 0.0f ? (sc.lo[0] - r.ox) * r.ix : INFINITY);
  const float tey = dy > 0.0f ? (sc.hi[1] - r.oy) * r.iy : (dy < 0.0f ? (sc.lo[1] - r.oy) * r.iy : INFINITY);
  const float tez = dz > 0.0f ? (sc.hi[2] - r.oz) * r.iz : (dz < 0.0f ? (sc.lo[2] - r.oz) * r.iz : INFINITY);
  te0 = fmaxf(tex, 0.0f);
  te1 = fmaxf(tey, 0.0f);
  te2 = fmaxf(tez, 0.0f);
}

__device__ inline void seg_begin(Trav& s, float dx, float dy, float dz, const DevScene& sc) {
  float te0, te1, te2;
  exit_dists(s.r, dx, dy, dz, sc, te0, te1, te2);
  s.t = fminf(fminf(te0, te1), te2);
  slab_margins(s.r, sc.wext);
  rotate_origin(s.r);
  s.idx = -1;
  s.oid = 0x7fffffff;
  s.node = 0;
  s.sp = 0;
}

__device__ inline void tri_candidate(Trav& s, const LaneScene& L, uint32_t k, uint32_t& tests) {
  // rotated record: V0, V1, V2 as five floats each (x, y, z, x, y), then the
  // caller's index; the ray's three coordinates start at byte 4 kx
  const GAS char* R = (const GAS char*)L.tris + ((size_t)k << 6);
  const GAS char* P = R + (s.r.kk & 0xFu);
  const GAS float* F = (const GAS float*)P;
  const float3 a = make_float3(F[0], F[1], F[2]), b = make_float3(F[5], F[6], F[7]),
               c = make_float3(F[10], F[11], F[12]);
  const int32_t oid = *(const GAS int32_t*)(R + 60);
  ++tests;
  float t, b1, b2;
  if (tri_test(s.r, a, b, c, s.t, t, b1, b2)) {
    // closest hit; equal distances go to the lower caller index
    if (t < s.t || (t == s.t && oid < s.oid)) {
      s.t = t;
      s.b1 = b1;
      s.b2 = b2;
      s.idx = (int32_t)k;
      s.oid = oid;
    }
  }
}

// Push onto the lane's stack: the first sd entries in LDS (lstk, stride 64
// words), the rest in global memory (gstk, stride 64 words).
__device__ inline bool push(Trav& s, LAS uint32_t* lstk, GAS uint32_t* gstk, int sd, int gd, uint32_t v) {
  if (s.sp < sd)
    lstk[s.sp * 64] = v;
  else if (s.sp < sd + gd)
    gstk[(s.sp - sd) * 64] = v;
  else
    return false;
  ++s.sp;
  return true;
}

__device__ inline void cswap(float& da, uint32_t& na, float& db, uint32_t& nb) {
  const bool sw = db < da;
  const float d = sw ? db : da;
  const uint32_t n = sw ? nb : na;
  db = sw ? da : db;
  nb = sw ? na : nb;
  da = d;
  na = n;
}

// One 4-wide node of the traversal.  Returns true when the segment's
// traversal has finished (stack empty).  Leaf children whose boxes the ray
// enters are tested at once (which can shorten the ray before the inner
// children are kept); the inner children hit are visited nearest first, the
// others pushed farthest first so they pop in order of entry distance.
__device__ inline bool trav_step(Trav& s, const LaneScene& L, LAS uint32_t* lstk, GAS uint32_t* gstk, int sd,
                                 int gd, uint32_t& visits, uint32_t& tests, bool& ovf) {
  const GAS f4v* N = (const GAS f4v*)L.nodes + 4 * (size_t)s.node;
  const f4v q0 = N[0], lk = N[1], q2 = N[2], q3 = N[3];
  ++visits;
  const RayP& r = s.r;
  // per axis: distance per code step (exact, the scale being a power of
  // two) and the near and far distances of the node origin with the margin
  const float ax = q0.w * r.ix, ay = q3.z * r.iy, az = q3.w * r.iz;
  const float bx = q0.x - r.ox, by = q0.y - r.oy, bz = q0.z - r.oz;
  const float mx = r.w * fabsf(r.ix), my = r.w * fabsf(r.iy), mz = r.w * fabsf(r.iz);
  const float nbx = fmaf(bx, r.ix, -mx), nby = fmaf(by, r.iy, -my), nbz = fmaf(bz, r.iz, -mz);
  const float fbx = fmaf(bx, r.ix, mx), fby = fmaf(by, r.iy, my), fbz = fmaf(bz, r.iz, mz);
  const uint32_t qlx = __float_as_uint(q2.x), qly = __float_as_uint(q2.y), qlz = __float_as_uint(q2.z),
                 qhx = __float_as_uint(q2.w), qhy = __float_as_uint(q3.x), qhz = __float_as_uint(q3.y);
  // per axis, the bound the ray enters through and the one it leaves through
  const bool px = r.ix >= 0.0f, py = r.iy >= 0.0f, pz = r.iz >= 0.0f;
  const uint32_t qnx = px ? qlx : qhx, qfx = px ? qhx : qlx, qny = py ? qly : qhy, qfy = py ? qhy : qly,
                 qnz = pz ? qlz : qhz, qfz = pz ? qhz : qlz;
#define QB(w, j) ((float)(((w) >> (8 * (j))) & 0xFFu))
#define CHILD_BOX(j)                                                                                           \
  fmaf(QB(qnx, j), ax, nbx), fmaf(QB(qny, j), ay, nby), fmaf(QB(qnz, j), az, nbz), fmaf(QB(qfx, j), ax, fbx), \
      fmaf(QB(qfy, j), ay, fby), fmaf(QB(qfz, j), az, fbz)
  float d0, d1, d2, d3;
  uint32_t c0 = __float_as_uint(lk.x), c1 = __float_as_uint(lk.y), c2 = __float_as_uint(lk.z),
           c3 = __float_as_uint(lk.w);
  bool h0 = box_hit(CHILD_BOX(0), s.t, d0) && c0 != kEmpty;
  bool h1 = box_hit(CHILD_BOX(1), s.t, d1) && c1 != kEmpty;
  bool h2 = box_hit(CHILD_BOX(2), s.t, d2) && c2 != kEmpty;
  bool h3 = box_hit(CHILD_BOX(3), s.t, d3) && c3 != kEmpty;
#undef QB
#undef CHILD_BOX
  // leaf children hit: one loop over the lane's own leaves, so the wave runs
  // as many triangle tests as its busiest lane rather than one per slot
  // that any lane needs
  uint32_t lm = (uint32_t)(h0 && (c0 & kLeafBit)) | ((uint32_t)(h1 && (c1 & kLeafBit)) << 1) |
                ((uint32_t)(h2 && (c2 & kLeafBit)) << 2) | ((uint32_t)(h3 && (c3 & kLeafBit)) << 3);
  h0 = h0 && !(lm & 1u);
  h1 = h1 && !(lm & 2u);
  h2 = h2 && !(lm & 4u);
  h3 = h3 && !(lm & 8u);
  while (lm) {
    const uint32_t j = (uint32_t)__builtin_ctz(lm);
    lm &= lm - 1u;
    const uint32_t cj = j == 0 ? c0 : (j == 1 ? c1 : (j == 2 ? c2 : c3));
    tri_candidate(s, L, cj & ~kLeafBit, tests);
  }
  // inner children entered before the (possibly shortened) closest hit
  d0 = h0 && d0 <= s.t ? d0 : INFINITY;
  d1 = h1 && d1 <= s.t ? d1 : INFINITY;
  d2 = h2 && d2 <= s.t ? d2 : INFINITY;
  d3 = h3 && d3 <= s.t ? d3 : INFINITY;
  const int cnt = (d0 < INFINITY) + (d1 < INFINITY) + (d2 < INFINITY) + (d3 < INFINITY);
  if (cnt == 0) {
    if (s.sp == 0) return true;
    --s.sp;
    s.node = s.sp < sd ? lstk[s.sp * 64] : gstk[(s.sp - sd) * 64];
    return false;
  }
  if (cnt > 1) {
    // sorting network on (distance, child), ascending; misses sort last
    cswap(d0, c0, d1, c1);
    cswap(d2, c2, d3, c3);
    cswap(d0, c0, d2, c2);
    cswap(d1, c1, d3, c3);
    cswap(d1, c1, d2, c2);
    if (s.sp + 3 <= sd) {
      // common case: three free LDS entries, so write all three (entries above
      // the new top are free) and move the top once; farthest lowest
      lstk[s.sp * 64] = cnt >= 4 ? c3 : (cnt == 3 ? c2 : c1);
      lstk[(s.sp + 1) * 64] = cnt >= 4 ? c2 : c1;
      lstk[(s.sp + 2) * 64] = c1;
      s.sp += cnt - 1;
    } else {
      bool ok = true;
      if (cnt >= 4) ok = ok && push(s, lstk, gstk, sd, gd, c3);
      if (cnt >= 3) ok = ok && push(s, lstk, gstk, sd, gd, c2);
      ok = ok && push(s, lstk, gstk, sd, gd, c1);
      if (!ok) {
        ovf = true;
        return true;
      }
    }
    s.node = c0;
    return false;
  }
  s.node = d0 < INFINITY ? c0 : (d1 < INFINITY ? c1 : (d2 < INFINITY ? c2 : c3));
  return false;
}

// End of a segment: returns the ray's outcome, or -1 when the ray re-enters
// through the opposite x / y face and traversal continues (section 2.2
// boundaries: periodic in x and y, substrate or open bottom at z_min,
// escape at z_max).
__device__ inline int seg_end(Trav& s, float dx, float dy, float dz, const DevScene& sc, bool ovf, float& px,
                              float& py) {
  if (s.idx >= 0) {
    s.total += s.t;
    return K_HIT;
  }
  const RayP& r = s.r;
  float te0, te1, te2;
  exit_dists(r, dx, dy, dz, sc, te0, te1, te2);
  if (te2 <= te0 && te2 <= te1) {
    s.total += te2;
    if (dz > 0.0f) return K_ESCAPE;
    if (sc.flags & 2u) {
      px = r.ox + te2 * dx;
      py = r.oy + te2 * dy;
      return K_SUBSTRATE;
    }
    return K_LOST;
  }
  const float texit = s.t;
  if (!(sc.flags & 1u) || ovf) {
    s.total += texit;
    return K_LOST;
  }
  s.total += texit;
  float qx = r.ox + texit * dx, qy = r.oy + texit * dy, qz = r.oz + texit * dz;
  if (te0 == texit)
    qx = dx > 0.0f ? sc.lo[0] : sc.hi[0];
  else
    qx = fminf(fmaxf(qx, sc.lo[0]), sc.hi[0]);
  if (te1 == texit)
    qy = dy > 0.0f ? sc.lo[1] : sc.hi[1];
  else
    qy = fminf(fmaxf(qy, sc.lo[1]), sc.hi[1]);
  qz = fminf(fmaxf(qz, sc.lo[2]), sc.hi[2]);
  s.r.ox = qx;
  s.r.oy = qy;
  s.r.oz = qz;
  if (++s.wraps > kWrapMax) return K_LOST;
  return -1;
}

// Primary ray of concatenated index g (Fig. flow: a uniform point of the top
// face, azimuth uniform, fixed or uniform polar angle).
__device__ inline void primary_ray(const DevJob& J, uint64_t g, float& ox, float& oy, float& oz, float& dx, float& dy,
                                   float& dz) {
  const uint64_t pid = J.pid0 + (g - J.gbase);
  const U4 u = philox(J.seed, (uint32_t)pid, (uint32_t)(pid >> 32), 0u, 0u);
  const float th = (J.theta >= 0.0f ? J.theta : -J.theta * u01(u.w)) * (kPi / 180.0f);
  const float psi = 2.0f * kPi * u01(u.z);
  ox = J.sc.lo[0] + (J.sc.hi[0] - J.sc.lo[0]) * u01(u.x);
  oy = J.sc.lo[1] + (J.sc.hi[1] - J.sc.lo[1]) * u01(u.y);
  oz = J.sc.hi[2];
  const float st = sinf(th);
  dx = st * cosf(psi);
  dy = st * sinf(psi);
  dz = -cosf(th);
}

extern __shared__ __align__(16) unsigned char smem[];

// Closest-hit traversal of one generation of rays.  A lane is idle, busy
// (traversing a segment) or finished (its segment's traversal is over).  The
// common iteration is one node step of the busy lanes; finished lanes are
// serviced together -- segment end, periodic re-entry, hit record -- and idle
// lanes take new rays once at least `refill` lanes are not busy.  So a wave is
// neither held by its slowest ray nor made to run the rare paths on every
// iteration.  Rays come from a per-wave reservation of consecutive indices,
// claimed from the generation's counter in guided blocks (a share of the
// estimated remaining work, at least the idle lanes, at most kClaimMax): one
// contended atomic serves many refills early on, and blocks shrink towards
// the end so the waves finish together.  MULTI: rays may belong to different jobs.
template <bool MULTI>
__device__ inline void traverse_body(const TraverseArgs& a) {
  const int wpb = blockDim.x >> 6;
  const int w = threadIdx.x >> 6;
  const uint32_t lane = lane_id();
  const uint64_t lt = (1ull << lane) - 1ull;
  LAS uint32_t* lstk = (LAS uint32_t*)smem + (size_t)w * a.lds_stack * 64 + lane;
  LAS float* ldir = (LAS float*)smem + (size_t)wpb * a.lds_stack * 64 + (size_t)w * 192 + lane;  // [3][64] per wave
  GAS uint32_t* gstk = gp(a.gstack) + ((size_t)(blockIdx.x * wpb + w) * a.gstack_depth) * 64 + lane;
  const uint32_t count = (a.src == 1 && a.count_in) ? min(*gp(a.count_in), a.qcap) : a.count;

  Trav s;
  LaneScene L;
  int job = 0;
  uint32_t item = 0, visits = 0, tests = 0;
  int st = 0;  // 0 idle, 1 busy, 2 finished
  bool ovf = false;
  bool exhausted = false;
  uint32_t res_lo = 0, res_hi = 0, seen = 0;  // wave-uniform reservation and counter estimate
  const uint32_t total_waves = gridDim.x * (uint32_t)wpb;
  if (!MULTI) {
    L.nodes = a.jobs[0].sc.nodes;
    L.tris = a.jobs[0].sc.tris_t;
    L.n_tris = a.jobs[0].sc.n_tris;
    L.flags = a.jobs[0].sc.flags;
  }
  for (;;) {
    const uint64_t busy = __ballot(st == 1);
    if (64u - (uint32_t)__popcll(busy) >= (uint32_t)a.refill || busy == 0ull) {
      if (st == 2) {
        float px = 0.f, py = 0.f;
        const DevScene& sc = a.jobs[job].sc;
        const float dx = ldir[0], dy = ldir[64], dz = ldir[128];
        const int kind = seg_end(s, dx, dy, dz, sc, ovf, px, py);
        if (kind < 0) {
          seg_begin(s, dx, dy, dz, sc);
          st = 1;
        } else {
          int32_t code;
          float f0 = s.b1, f1 = s.b2;
          if (kind == K_HIT) {
            code = s.idx;
          } else if (kind == K_ESCAPE) {
            code = -1;
          } else if (kind == K_SUBSTRATE) {
            code = -2;
            f0 = px;
            f1 = py;
          } else {
            code = -3;
          }
          gp(a.hit.code)[item] = code;
          gp(a.hit.f0)[item] = f0;
          gp(a.hit.f1)[item] = f1;
          gp(a.hit.t)[item] = s.total;
          gp(a.hit.visits)[item] = visits;
          gp(a.hit.tests)[item] = tests;
          gp(a.hit.wraps)[item] = (uint32_t)s.wraps | (ovf ? 0x80000000u : 0u);
          if (ovf) atomicOr(a.err, 2u);
          st = 0;
        }
      }
      const uint64_t idle = __ballot(st == 0);
      if (idle && (res_lo < res_hi || !exhausted)) {
        const uint32_t nidle = (uint32_t)__popcll(idle);
        const uint32_t have = res_hi - res_lo;
        uint32_t base = 0, new_hi = 0;
        bool claimed = false;
        if (have < nidle && !exhausted) {
          const uint32_t want = nidle - have;
          const uint32_t left = count > seen ? count - seen : 0u;
          uint32_t claim = (left / (2u * total_waves)) & ~63u;
          claim = claim > (uint32_t)kClaimMax ? (uint32_t)kClaimMax : claim;
          claim = claim < want ? want : claim;
          if (lane == 0) base = __hip_atomic_fetch_add(gp(a.work), claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          base = __builtin_amdgcn_readlane(base, 0);  // lane 0's claim, wave-uniform (scalar registers)
          seen = base + claim;
          if (base + claim >= count) exhausted = true;
          new_hi = base >= count ? base : min(base + claim, count);
          claimed = true;
        }
        const uint32_t rank = (uint32_t)__popcll(idle & lt);
        if (st == 0) {
          bool got = false;
          if (rank < have) {
            item = res_lo + rank;
            got = true;
          } else if (claimed) {
            item = base + (rank - have);
            got = item < new_hi;
          }
          if (got) {
            float ox, oy, oz, dx, dy, dz;
            if (a.src == 1) {
              ox = gp(a.qin.ox)[item];
              oy = gp(a.qin.oy)[item];
              oz = gp(a.qin.oz)[item];
              dx = gp(a.qin.dx)[item];
              dy = gp(a.qin.dy)[item];
              dz = gp(a.qin.dz)[item];
              if (MULTI) job = (int)(gp(a.qin.meta)[item] >> 4);
            } else {
              const GAS float* q = gp(a.rays) + 6 * (size_t)item;
              ox = q[0];
              oy = q[1];
              oz = q[2];
              dx = q[3];
              dy = q[4];
              dz = q[5];
            }
            if (MULTI) {
              L.nodes = a.jobs[job].sc.nodes;
              L.tris = a.jobs[job].sc.tris_t;
              L.n_tris = a.jobs[job].sc.n_tris;
              L.flags = a.jobs[job].sc.flags;
            }
            ray_setup(s.r, dx, dy, dz);
            s.r.ox = ox;
            s.r.oy = oy;
            s.r.oz = oz;
            s.total = 0.0f;
            s.wraps = 0;
            visits = 0;
            tests = 0;
            ovf = false;
            ldir[0] = dx;
            ldir[64] = dy;
            ldir[128] = dz;
            seg_begin(s, dx, dy, dz, a.jobs[job].sc);
            st = 1;
          }
        }
        if (claimed) {
          const uint32_t lo2 = base + (nidle - have);
          res_lo = lo2 < new_hi ? lo2 : new_hi;
          res_hi = new_hi;
        } else {
          res_lo = res_lo + nidle < res_hi ? res_lo + nidle : res_hi;
        }
      }
      // after servicing no lane is finished: none busy means the work is done
      if (__ballot(st == 1) == 0ull) break;
    }
    if (st == 1) {
      if (L.n_tris == 0 || trav_step(s, L, lstk, gstk, a.lds_stack, a.gstack_depth, visits, tests, ovf)) st = 2;
    }
  }
}

// Register-limited builds: k_traverse caps registers for 7 waves per SIMD
// (72 VGPRs; no spills for one scene, a few for the batched form); O6 caps
// them for 6 waves (80 VGPRs, no spills in either form) and O8 for 8 waves at
// the price of more spilled, rarely used values.  One scene runs the 7-wave
// build unless 6 or 8 waves are asked for; a batch runs the 6-wave build
// unless 8 are (its 7-wave form spills).  The autotuner picks by measurement.
template <bool MULTI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) void k_traverse(TraverseArgs a) {
  traverse_body<MULTI>(a);
}

template <bool MULTI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_traverse_o6(TraverseArgs a) {
  traverse_body<MULTI>(a);
}

template <bool MULTI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_traverse_o8(TraverseArgs a) {
  traverse_body<MULTI>(a);
}

// Primary rays of one chunk, written to the queue so that both launches of
// generation 0 read them like any other generation.
__global__ void k_primaries(const DevJob* __restrict__ jobs, int32_t j_lo, int32_t j_hi, uint64_t chunk_lo,
                            uint32_t n, RayQueue q) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint64_t g = chunk_lo + i;
    const int job = find_job(jobs, j_lo, j_hi, g);
    float ox, oy, oz, dx, dy, dz;
    primary_ray(jobs[job], g, ox, oy, oz, dx, dy, dz);
    gp(q.ox)[i] = ox;
    gp(q.oy)[i] = oy;
    gp(q.oz)[i] = oz;
    gp(q.dx)[i] = dx;
    gp(q.dy)[i] = dy;
    gp(q.dz)[i] = dz;
    gp(q.E)[i] = jobs[job].E0;
    gp(q.path)[i] = 0u;
    gp(q.ci)[i] = i;
    gp(q.meta)[i] = (uint32_t)job << 4;
  }
}

// Hit records -> caller triangle indices (first-hit entry point).
__global__ void k_hit_ids(const float4* __restrict__ tris, const int32_t* __restrict__ code, int64_t n,
                          int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t c = code[i];
  out[i] = c >= 0 ? (int32_t)__float_as_uint(tris[3 * (size_t)c].w) : c;
}

// Shading of one generation (section 2.2): for every ray, its hit record
// decides escape, absorption or emission; emitting hits draw the daughter
// count, energies and directions and append the daughters to the next queue
// with one atomic per workgroup step.  Tables sit in LDS; counters
// accumulate in per-lane registers for the wave's current job (flushed when
// it changes), histograms in per-wave LDS blocks, or everything in per-job
// LDS blocks when the chunk holds few jobs.
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4))) void k_shade(ShadeArgs a) {
  const int wpb = blockDim.x >> 6;
  const int w = threadIdx.x >> 6;
  const uint32_t lane = lane_id();
  const DevTables& tb = a.tb;
  const int nY = tb.nE * tb.nth;
  LAS unsigned char* lds = (LAS unsigned char*)smem;
  LAS float* s_yld = (LAS float*)lds;
  LAS float* s_cE = s_yld + nY;
  LAS float* s_cF = s_cE + tb.ncdf;
  LAS uint16_t* s_gF = (LAS uint16_t*)(s_cF + tb.ncdf);
  LAS uint16_t* s_gE = s_gF + kGuide;
  size_t off = ((size_t)(nY + 2 * tb.ncdf) * 4 + 4 * kGuide + 15) & ~(size_t)15;
  LAS uint32_t* s_eh = (LAS uint32_t*)(lds + off);
  LAS uint32_t* s_ah = s_eh + wpb * a.n_ebins;
  LAS uint32_t* s_zh = s_ah + wpb * a.n_abins;
  __shared__ uint32_t s_wtot[16], s_wbase[16];  // per-wave daughter totals and queue offsets of a step
  JobTab jtab;
  jtab.base = lds + off;
  jtab.stride = (T_NCOUNT * 8 + (a.n_ebins + a.n_abins + a.n_zbins) * 4 + 7) & ~7;
  jtab.n_eb = a.n_ebins;
  jtab.n_ab = a.n_abins;
  jtab.j_lo = a.j_lo;
  jtab.J = a.j_hi - a.j_lo + 1;
  const bool shared = jtab.J <= kShadeJobs;
  const JobTab* jt = shared ? &jtab : nullptr;

  const uint32_t count = a.gen == 0 ? a.n_gen0 : min(*gp(a.count_in), a.qcap);  // queue length
  // each workgroup takes one contiguous slice (a multiple of its size), in
  // steps of blockDim.x rays, 64 per wave: neighbouring rays mostly share a
  // job, so the per-wave tallies rarely change owner, and the workgroup
  // reserves queue space for its daughters with one atomic per step
  const uint32_t per = ((count + gridDim.x - 1) / gridDim.x + blockDim.x - 1) / blockDim.x * blockDim.x;
  const uint64_t wg0 = (uint64_t)blockIdx.x * per;
  if (wg0 >= count) return;  // whole workgroup idle
  const uint32_t wg1 = (uint32_t)min((uint64_t)count, wg0 + per);
  for (int i = threadIdx.x; i < nY; i += blockDim.x) s_yld[i] = gp(tb.yld)[i];
  for (int i = threadIdx.x; i < tb.ncdf; i += blockDim.x) {
    s_cE[i] = gp(tb.cdfE)[i];
    s_cF[i] = gp(tb.cdfF)[i];
  }
  for (int i = threadIdx.x; i < kGuide; i += blockDim.x) {
    s_gF[i] = gp(tb.gF)[i];
    s_gE[i] = gp(tb.gE)[i];
  }
  if (shared) {
    const int words = jtab.J * jtab.stride / 4;
    for (int i = threadIdx.x; i < words; i += blockDim.x) ((LAS uint32_t*)jtab.base)[i] = 0u;
  } else {
    for (int i = threadIdx.x; i < wpb * a.n_ebins; i += blockDim.x) s_eh[i] = 0u;
    for (int i = threadIdx.x; i < wpb * a.n_abins; i += blockDim.x) s_ah[i] = 0u;
    for (int i = threadIdx.x; i < wpb * a.n_zbins; i += blockDim.x) s_zh[i] = 0u;
  }
  __syncthreads();

  WaveTally wt;
#pragma unroll
  for (int k = 0; k < T_NCOUNT; ++k) wt.c[k] = 0u;
  wt.e_esc = 0ull;
  wt.e_dep = 0ull;
  wt.eh = s_eh + w * a.n_ebins;
  wt.ah = s_ah + w * a.n_abins;
  wt.zh = s_zh + w * a.n_zbins;
  int tag = -1;
  for (uint32_t step = (uint32_t)wg0; step < wg1; step += blockDim.x) {
    const uint32_t base = step + (uint32_t)w * 64u;
    const uint32_t item = base + lane;
    const bool active = item < wg1;

    float ox = 0.f, oy = 0.f, oz = 0.f, dx = 0.f, dy = 0.f, dz = -1.f, E = 0.f;
    uint32_t path = 0, ci = 0;
    int gen = a.gen, job = 0;
    if (active) {
      {
        dx = gp(a.qin.dx)[item];
        dy = gp(a.qin.dy)[item];
        dz = gp(a.qin.dz)[item];
        E = gp(a.qin.E)[item];
        path = gp(a.qin.path)[item];
        ci = gp(a.qin.ci)[item];
        const uint32_t m = gp(a.qin.meta)[item];
        gen = (int)(m & 15u);
        job = (int)(m >> 4);
      }
    }
    (void)ox;
    (void)oy;
    (void)oz;
    const int j0 = __builtin_amdgcn_readlane(job, 0);
    if (base < wg1 && j0 != tag) {  // lane 0 active: the wave has rays this step
      if (tag >= 0) {
        if (shared)
          flush_wave_lds(wt, jt_cnt(jtab, tag), lane);
        else
          flush_wave(wt, a.jobs[tag].tally, a.n_ebins, a.n_abins, a.n_zbins, lane);
      }
      tag = j0;
    }
    const DevJob& J = a.jobs[job];
    const bool mine = job == tag;
    unsigned long long* gt = J.tally;

    int nd = 0;
    float alpha = 0.f;
    float px = 0.f, py = 0.f, pz = 0.f, nx = 0.f, ny = 0.f, nz = 1.f;
    if (active) {
      const int32_t code = gp(a.hit.code)[item];
      const float f0 = gp(a.hit.f0)[item], f1 = gp(a.hit.f1)[item];
      const uint32_t wr = gp(a.hit.wraps)[item];
      tally_cnt(mine, wt, gt, T_RAYS, 1ull, jt, job);
      tally_cnt(mine, wt, gt, T_VISITS, gp(a.hit.visits)[item], jt, job);
      tally_cnt(mine, wt, gt, T_TESTS, gp(a.hit.tests)[item], jt, job);
      if (wr & 0x7fffffffu) tally_cnt(mine, wt, gt, T_WRAPS, (unsigned long long)(wr & 0x7fffffffu), jt, job);
      if (wr & 0x80000000u) tally_cnt(mine, wt, gt, T_STACKOVF, 1ull, jt, job);
      if (code == -1) {
        tally_cnt(mine, wt, gt, T_ESCAPED, 1ull, jt, job);
        tally_cnt(mine, wt, gt, T_E_ESC_FX, (unsigned long long)to_fx(E), jt, job);
        int eb = (int)floorf(E / J.E0 * (float)a.n_ebins);
        eb = min(max(eb, 0), a.n_ebins - 1);
        const float pol = acosf(fminf(dz, 1.0f)) * kDeg;
        int ab = (int)floorf(pol * (1.0f / 90.0f) * (float)a.n_abins);
        ab = min(max(ab, 0), a.n_abins - 1);
        if (shared) {
          LAS uint32_t* h = jt_eh(jtab, job);
          ladd(h + eb, 1u);
          ladd(h + a.n_ebins + ab, 1u);
        } else if (mine) {
          ladd(wt.eh + eb, 1u);
          ladd(wt.ah + ab, 1u);
        } else {
          gadd(gt + T_NCOUNT + eb, 1ull);
          gadd(gt + T_NCOUNT + a.n_ebins + ab, 1ull);
        }
        __hip_atomic_fetch_add(gp(a.ppc) + ci, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if (code == -3) {
        tally_cnt(mine, wt, gt, T_LOST, 1ull, jt, job);
        tally_cnt(mine, wt, gt, T_E_DEP_FX, (unsigned long long)to_fx(E), jt, job);
      } else {
        if (code == -2) {
          tally_cnt(mine, wt, gt, T_SUBSTRATE, 1ull, jt, job);
          px = f0;
          py = f1;
          pz = J.sc.lo[2];
        } else {
          const GAS f4v* T = (const GAS f4v*)J.sc.tris + 3 * (size_t)code;
          const f4v v0 = T[0], v1 = T[1], v2 = T[2];
          const float b1 = f0, b2 = f1, b0 = 1.0f - b1 - b2;
          px = b0 * v0.x + b1 * v1.x + b2 * v2.x;
          py = b0 * v0.y + b1 * v1.y + b2 * v2.y;
          pz = b0 * v0.z + b1 * v1.z + b2 * v2.z;
          const float e1x = v1.x - v0.x, e1y = v1.y - v0.y, e1z = v1.z - v0.z;
          const float e2x = v2.x - v0.x, e2y = v2.y - v0.y, e2z = v2.z - v0.z;
          const float sx = e1y * e2z - e1z * e2y, sy = e1z * e2x - e1x * e2z, sz = e1x * e2y - e1y * e2x;
          const float l2 = sx * sx + sy * sy + sz * sz;
          if (l2 > 1e-30f && l2 < 1e30f) {
            const float il = 1.0f / sqrtf(l2);
            nx = sx * il;
            ny = sy * il;
            nz = sz * il;
          } else {  // sliver: the FP32 cross product under- or overflows
            const double ax = (double)v1.x - v0.x, ay = (double)v1.y - v0.y, az = (double)v1.z - v0.z;
            const double bx = (double)v2.x - v0.x, by = (double)v2.y - v0.y, bz = (double)v2.z - v0.z;
            const double qx = ay * bz - az * by, qy = az * bx - ax * bz, qz = ax * by - ay * bx;
            const double il = 1.0 / sqrt(qx * qx + qy * qy + qz * qz);
            nx = (float)(qx * il);
            ny = (float)(qy * il);
            nz = (float)(qz * il);
          }
        }
        if (a.n_zbins > 0) {
          // the ray ends on a surface: its depth below the top of the cell, as
          // a fraction of the cell height (section 3.2, Fig. pen, penetration profile)
          int zb = (int)floorf((J.sc.hi[2] - pz) / (J.sc.hi[2] - J.sc.lo[2]) * (float)a.n_zbins);
          zb = min(max(zb, 0), a.n_zbins - 1);
          if (shared)
            ladd(jt_eh(jtab, job) + a.n_ebins + a.n_abins + zb, 1u);
          else if (mine)
            ladd(wt.zh + zb, 1u);
          else
            gadd(gt + T_NCOUNT + a.n_ebins + a.n_abins + zb, 1ull);
        }
        if (gen >= a.max_gen) {
          tally_cnt(mine, wt, gt, T_TRUNCATED, 1ull, jt, job);
          tally_cnt(mine, wt, gt, T_E_DEP_FX, (unsigned long long)to_fx(E), jt, job);
        } else {
          tally_cnt(mine, wt, gt, T_ABSORBED, 1ull, jt, job);
          if (E <= tb.Ec) {
            tally_cnt(mine, wt, gt, T_E_DEP_FX, (unsigned long long)to_fx(E), jt, job);
          } else {
            const float cosa = fminf(fmaxf(-(dx * nx + dy * ny + dz * nz), 0.0f), 1.0f);
            alpha = acosf(cosa) * kDeg;
            const float delta = table_yield(s_yld, tb, E, alpha);
            const uint64_t pid = J.pid0 + (a.chunk_lo + ci - J.gbase);
            const U4 u = philox(J.seed, (uint32_t)pid, (uint32_t)(pid >> 32), path, 1u);
            const float fl = floorf(delta);
            nd = (int)fl + (u01(u.x) < delta - fl ? 1 : 0);
            if (nd == 0) tally_cnt(mine, wt, gt, T_E_DEP_FX, (unsigned long long)to_fx(E), jt, job);
          }
        }
      }
    }

    // ---- daughters: one queue reservation per workgroup step
    const uint32_t incl = wave_incl_scan((uint32_t)nd, lane);
    if (lane == 63) s_wtot[w] = incl;
    __syncthreads();
    if (w == 0) {
      const uint32_t v = lane < (uint32_t)wpb ? s_wtot[lane] : 0u;
      const uint32_t inc2 = wave_incl_scan(v, lane);
      const uint32_t T = __builtin_amdgcn_readlane(inc2, 63);
      uint32_t b = 0;
      if (lane == 0 && T) b = __hip_atomic_fetch_add(gp(a.count_out), T, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      b = __builtin_amdgcn_readlane(b, 0);
      if (lane < (uint32_t)wpb) s_wbase[lane] = b + inc2 - v;
    }
    __syncthreads();
    const uint32_t obase = s_wbase[w];
    if (nd > 0) {
      const uint32_t first = obase + incl - (uint32_t)nd;
      const uint64_t pid = J.pid0 + (a.chunk_lo + ci - J.gbase);
      float Eav = E;
      long long fx_left = to_fx(E);
      float3 t1, t2;
      onb(nx, ny, nz, t1, t2);
      const float Lx = J.sc.hi[0] - J.sc.lo[0], Ly = J.sc.hi[1] - J.sc.lo[1];
      const bool periodic = (J.sc.flags & 1u) != 0;
      uint32_t dropped = 0;
      // the paper's rule: E_SEE at (E, alpha); a pair shares one xi
      const bool paper = tb.emission == kEmitPaper;
      const float es = paper ? table_yield((const GAS float*)tb.esee, tb, E, alpha) : 0.0f;
      float xi_pair = 0.0f;
      for (int d = 0; d < nd; ++d) {
        const U4 u = philox(J.seed, (uint32_t)pid, (uint32_t)(pid >> 32), path, 2u + (uint32_t)d);
        float Ed, xb;  // energy and sin^2 of the angle from the normal
        if (!paper) {
          Ed = cdf_inv(s_cE, s_cF, tb.ncdf, s_gF,
                       u01(u.x) * cdf_at(s_cE, s_cF, tb.ncdf, s_gE, tb.e1bits, tb.eshift, Eav));
          xb = u01(u.y);
        } else if (d & 1) {  // second of a pair: beta2 = pi/2 - beta1, E2 = cos^2(beta1) E_SEE
          Ed = (1.0f - xi_pair) * es;
          xb = 1.0f - xi_pair;
        } else if (d + 1 < nd) {  // first of a pair: E1 = E_SEE sqrt(xi), beta1 = asin(sqrt(xi))
          xi_pair = u01(u.y);
          Ed = es * sqrtf(xi_pair);
          xb = xi_pair;
        } else {  // a lone daughter
          Ed = es;
          xb = u01(u.y);
        }
        Ed = fminf(fmaxf(Ed, 0.0f), Eav);
        Eav -= Ed;
        fx_left -= to_fx(Ed);
        const float sb = sqrtf(xb), cb = sqrtf(1.0f - xb);
        const float ph = 2.0f * kPi * u01(u.z);
        const float cp = cosf(ph), sp = sinf(ph);
        const float ddx = cb * nx + sb * (cp * t1.x + sp * t2.x);
        const float ddy = cb * ny + sb * (cp * t1.y + sp * t2.y);
        const float ddz = cb * nz + sb * (cp * t1.z + sp * t2.z);
        float qx = px + kSpawnEps * nx, qy = py + kSpawnEps * ny, qz = pz + kSpawnEps * nz;
        if (periodic) {
          if (qx > J.sc.hi[0]) qx -= Lx;
          if (qx < J.sc.lo[0]) qx += Lx;
          if (qy > J.sc.hi[1]) qy -= Ly;
          if (qy < J.sc.lo[1]) qy += Ly;
        }
        qz = fminf(fmaxf(qz, J.sc.lo[2]), J.sc.hi[2]);
        const uint32_t slot = first + (uint32_t)d;
        if (slot < a.qcap) {
          gp(a.qout.ox)[slot] = qx;
          gp(a.qout.oy)[slot] = qy;
          gp(a.qout.oz)[slot] = qz;
          gp(a.qout.dx)[slot] = ddx;
          gp(a.qout.dy)[slot] = ddy;
          gp(a.qout.dz)[slot] = ddz;
          gp(a.qout.E)[slot] = Ed;
          gp(a.qout.path)[slot] = path * 8u + (uint32_t)d + 1u;
          gp(a.qout.ci)[slot] = ci;
          gp(a.qout.meta)[slot] = (uint32_t)(gen + 1) | ((uint32_t)job << 4);
        } else {
          ++dropped;
        }
      }
      tally_cnt(mine, wt, gt, T_E_DEP_FX, (unsigned long long)fx_left, jt, job);
      tally_cnt(mine, wt, gt, T_SPAWNED, (unsigned long long)nd, jt, job);
      if (dropped) {
        tally_cnt(mine, wt, gt, T_DROPPED, dropped, jt, job);
        atomicOr(a.err, 1u);
      }
    }
  }
  if (shared) {
    if (tag >= 0) flush_wave_lds(wt, jt_cnt(jtab, tag), lane);
    __syncthreads();
    // the workgroup's job blocks to global memory, nonzero entries only
    const int slots = T_NCOUNT + a.n_ebins + a.n_abins + a.n_zbins;
    for (int i = threadIdx.x; i < jtab.J * slots; i += blockDim.x) {
      const int j = i / slots, k = i % slots;
      const LAS unsigned char* blk = jtab.base + (size_t)j * jtab.stride;
      const unsigned long long v = k < T_NCOUNT
                                       ? ((const LAS unsigned long long*)blk)[k]
                                       : (unsigned long long)((const LAS uint32_t*)(blk + T_NCOUNT * 8))[k - T_NCOUNT];
      if (v) gadd(a.jobs[jtab.j_lo + j].tally + k, v);
    }
  } else if (tag >= 0) {
    flush_wave(wt, a.jobs[tag].tally, a.n_ebins, a.n_abins, a.n_zbins, lane);
  }
}

// Sum over the chunk's primaries of (escape count)^2 for the yield's standard
// error, and the optional per-primary output.  Each wave takes a contiguous
// slice of the chunk, so its items change job rarely: lanes accumulate in
// registers and the wave reduces once per job it touches.  The workgroup's
// waves then combine their sums for the job of its last item in LDS, so a
// single-job chunk costs one atomic per workgroup on the job's counter.
__global__ __launch_bounds__(256) void k_chunk_reduce(const DevJob* jobs, int32_t j_lo, int32_t j_hi,
                                                      const uint32_t* __restrict__ ppc, uint32_t n,
                                                      uint64_t chunk_lo) {
  __shared__ unsigned long long s_sum[4];
  __shared__ int s_job[4];
  const uint32_t lane = lane_id();
  const uint32_t w = threadIdx.x >> 6;
  const uint32_t wpb = blockDim.x >> 6;
  const uint32_t total_waves = gridDim.x * wpb;
  const uint64_t per = (((uint64_t)n + total_waves - 1) / total_waves + 63) & ~63ull;
  const uint64_t b = (uint64_t)(blockIdx.x * wpb + w) * per;
  int tag = -1;
  unsigned long long acc = 0;
  if (b < n) {
    const uint32_t e = (uint32_t)(b + per < n ? b + per : n);
    tag = find_job(jobs, j_lo, j_hi, chunk_lo + b);
    uint64_t end = tag < j_hi ? gp(jobs)[tag + 1].gbase : ~0ull;
    uint32_t* pp = gp(jobs)[tag].pp_escaped;
    uint64_t pbase = gp(jobs)[tag].gbase;
    for (uint32_t i4 = (uint32_t)b; i4 < e; i4 += 256) {
      // four loads in flight per lane, then the items in order
      uint32_t cv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t i = i4 + 64u * k + lane;
        cv[k] = i < e ? gp(ppc)[i] : 0u;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t i0 = i4 + 64u * k;
        if (i0 >= e) break;
        const uint32_t i = i0 + lane;
        const bool ok = i < e;
        const uint64_t g = chunk_lo + i;
        const uint32_t c = cv[k];
        const uint64_t g_last = chunk_lo + (i0 + 63 < e ? i0 + 63 : e - 1);
        if (g_last < end) {
          acc += (unsigned long long)c * c;
          if (pp && ok) gp(pp)[g - pbase] = c;
        } else {
          // the wave's items reach into later jobs
          const int j = ok ? find_job(jobs, tag, j_hi, g) : tag;
          if (j == tag)
            acc += (unsigned long long)c * c;
          else if (c)
            gadd(&jobs[j].tally[T_C2], (unsigned long long)c * c);
          uint32_t* pj = gp(jobs)[j].pp_escaped;
          if (pj && ok) gp(pj)[g - gp(jobs)[j].gbase] = c;
          const unsigned long long sum = wave_sum(acc);
          if (lane == 0 && sum) gadd(&jobs[tag].tally[T_C2], sum);
          acc = 0;
          tag = find_job(jobs, tag, j_hi, g_last);
          end = tag < j_hi ? gp(jobs)[tag + 1].gbase : ~0ull;
          pp = gp(jobs)[tag].pp_escaped;
          pbase = gp(jobs)[tag].gbase;
        }
      }
    }
  }
  const unsigned long long sum = wave_sum(acc);
  if (lane == 0) {
    s_sum[w] = sum;
    s_job[w] = tag;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // waves with the same final job add together (the slices are in order)
    unsigned long long run = 0;
    int cur = -1;
    for (uint32_t k = 0; k < wpb; ++k) {
      if (s_job[k] != cur) {
        if (cur >= 0 && run) gadd(&jobs[cur].tally[T_C2], run);
        cur = s_job[k];
        run = 0;
      }
      run += s_sum[k];
    }
    if (cur >= 0 && run) gadd(&jobs[cur].tally[T_C2], run);
  }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// Streaming copy used to measure achievable HBM bandwidth: four independent
// 16-byte loads in flight per lane, coalesced across the wave.
__global__ __launch_bounds__(256) void k_copy_probe(float4* __restrict__ dst4, const float4* __restrict__ src4,
                                                    size_t n) {
  const f4v* src = reinterpret_cast<const f4v*>(src4);
  f4v* dst = reinterpret_cast<f4v*>(dst4);
  const size_t stride = (size_t)gridDim.x * 1024;
  for (size_t base = (size_t)blockIdx.x * 1024 + threadIdx.x; base < n; base += stride) {
    f4v v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const size_t i = base + (size_t)j * 256;
      if (i < n) v[j] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const size_t i = base + (size_t)j * 256;
      if (i < n) __builtin_nontemporal_store(v[j], dst + i);
    }
  }
}

}  // namespace

// per wave: the stacks' LDS part, then the lanes' ray directions
size_t traverse_lds_bytes(int lds_stack, int block) { return (size_t)(block / 64) * (lds_stack + 3) * 64 * 4; }

size_t shade_lds_bytes(const DevTables& tb, int n_hist, int block, int n_jobs) {
  const int wpb = block / 64;
  size_t off = ((size_t)(tb.nE * tb.nth + 2 * tb.ncdf) * 4 + 4 * kGuide + 15) & ~(size_t)15;
  const size_t per_wave = (size_t)wpb * n_hist * 4;
  const size_t per_job = n_jobs <= kShadeJobs
                             ? (size_t)n_jobs * ((T_NCOUNT * 8 + n_hist * 4 + 7) & ~7)
                             : 0;
  return off + (per_wave > per_job ? per_wave : per_job);
}

hipError_t launch_traverse(const TraverseArgs& a, bool multi, int occupancy, int grid, int block, hipStream_t s) {
  const size_t lds = traverse_lds_bytes(a.lds_stack, block);
  // waves per SIMD of the build: 8 or 6 when asked, else 7 for one scene and
  // 6 for a batch
  const int w = occupancy >= 8 ? 8 : (occupancy == 6 || multi ? 6 : 7);
  if (w == 8) {
    if (multi)
      k_traverse_o8<true><<<grid, block, lds, s>>>(a);
    else
      k_traverse_o8<false><<<grid, block, lds, s>>>(a);
  } else if (w == 6) {
    if (multi)
      k_traverse_o6<true><<<grid, block, lds, s>>>(a);
    else
      k_traverse_o6<false><<<grid, block, lds, s>>>(a);
  } else {
    k_traverse<false><<<grid, block, lds, s>>>(a);
  }
  return hipGetLastError();
}

hipError_t launch_shade(const ShadeArgs& a, int n_cu, int block, hipStream_t s) {
  const size_t lds = shade_lds_bytes(a.tb, a.n_ebins + a.n_abins + a.n_zbins, block, a.j_hi - a.j_lo + 1);
  // every workgroup resident at once: the waves take equal contiguous slices,
  // so a second round of workgroups would double the kernel's time
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_shade, block, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  k_shade<<<n_cu * per_cu, block, lds, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_primaries(const DevJob* jobs, int32_t j_lo, int32_t j_hi, uint64_t chunk_lo, uint32_t n,
                            const RayQueue& q, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int grid = (int)((n + 255) / 256);
  if (grid > 16384) grid = 16384;
  k_primaries<<<grid, 256, 0, s>>>(jobs, j_lo, j_hi, chunk_lo, n, q);
  return hipGetLastError();
}

hipError_t launch_hit_ids(const float4* tris, const int32_t* code, int64_t n, int32_t* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_hit_ids<<<(int)((n + 255) / 256), 256, 0, s>>>(tris, code, n, out);
  return hipGetLastError();
}

hipError_t launch_chunk_reduce(const DevJob* jobs, int32_t j_lo, int32_t j_hi, const uint32_t* ppc, uint32_t n,
                               uint64_t chunk_lo, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int grid = (int)((n + 255) / 256);
  if (grid > 1024) grid = 1024;
  k_chunk_reduce<<<grid, 256, 0, s>>>(jobs, j_lo, j_hi, ppc, n, chunk_lo);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  k_fill_u32<<<(int)g, 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  k_fill_u64<<<(int)g, 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

hipError_t launch_copy_probe(float4* dst, const float4* src, size_t n16, int grid, hipStream_t s) {
  k_copy_probe<<<grid, 256, 0, s>>>(dst, src, n16);
  return hipGetLastError();
}

}  // namespace rtmc
