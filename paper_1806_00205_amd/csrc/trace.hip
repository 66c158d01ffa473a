// Ray tracing Monte Carlo on gfx950: one lane per ray.
//
// A generation of rays (the paper's tree of branches, section 2.2, handled
// breadth-first across all primaries) is processed by two launches:
//   k_traverse: closest front-facing triangle by BVH traversal (section 2.1):
//     robust slab tests against both child boxes of a 64-byte node record and
//     the watertight ray/triangle test of Woop, Benthin and Wald (JCGT 2013)
//     with back-face culling; periodic re-entry through the x / y faces,
//     escape through z_max, substrate plane at z_min (section 2.2).  Lanes
//     whose ray is done fetch new rays, so waves stay full.  Output: one
//     28-byte hit record per ray.
//   k_shade: the local incidence angle and the flat-surface tables give the
//     daughter count (stochastic rounding, footnote of section 2.2), energies
//     (inverse of the tabulated CDF truncated to the energy still available)
//     and cosine-law directions; daughters are appended to the next queue with
//     one atomic per wave; tallies go to per-wave LDS blocks.
// Generation 0 rays are regenerated from primary ids in both launches rather
// than stored.  Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed
// by the job seed, counter (primary id, 0, path code, draw); draw 0 = birth
// of a primary, 1 = daughter count, 2 + d = daughter d; a daughter's path
// code is parent * 8 + d + 1.
#include "rtmc_internal.h"

namespace rtmc {
namespace {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kDeg = 57.295779513082320876f;  // 180 / pi
constexpr float kRobust = 1.0000004f;  // >= 1 + 2 gamma(3): conservative far slab distance

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

struct RayP {
  float ox, oy, oz, dx, dy, dz;
  float ix, iy, iz;
  float Sx, Sy, Sz;
  int kx, ky, kz;
};

__device__ inline float pick(float x, float y, float z, int k) { return k == 0 ? x : (k == 1 ? y : z); }

__device__ inline float safe_inv(float d) { return 1.0f / (fabsf(d) > 1e-20f ? d : copysignf(1e-20f, d)); }

__device__ inline void ray_setup(RayP& r, float dx, float dy, float dz) {
  r.dx = dx;
  r.dy = dy;
  r.dz = dz;
  r.ix = safe_inv(dx);
  r.iy = safe_inv(dy);
  r.iz = safe_inv(dz);
  const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
  int kz = ax > ay ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
  int kx = kz == 2 ? 0 : kz + 1;
  int ky = kx == 2 ? 0 : kx + 1;
  const float dkz = pick(dx, dy, dz, kz);
  if (dkz < 0.0f) {
    int t = kx;
    kx = ky;
    ky = t;
  }
  r.kx = kx;
  r.ky = ky;
  r.kz = kz;
  r.Sx = pick(dx, dy, dz, kx) / dkz;
  r.Sy = pick(dx, dy, dz, ky) / dkz;
  r.Sz = 1.0f / dkz;
}

__device__ inline bool box_test(const RayP& r, float lx, float ly, float lz, float hx, float hy, float hz, float tmax,
                                float& tn) {
  const float tx0 = (lx - r.ox) * r.ix, tx1 = (hx - r.ox) * r.ix;
  const float ty0 = (ly - r.oy) * r.iy, ty1 = (hy - r.oy) * r.iy;
  const float tz0 = (lz - r.oz) * r.iz, tz1 = (hz - r.oz) * r.iz;
  const float t0 = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
  const float t1 = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1)) * kRobust;
  tn = t0;
  return t0 <= fminf(t1, tmax);
}

// Watertight ray/triangle test with back-face culling.  U, V, W are the
// sheared edge functions (weights of V0, V1, V2); products are kept
// unfused so that an edge shared by two triangles gets exactly opposite
// values, and an exactly zero edge function is recomputed in FP64.
__device__ inline bool tri_test(const RayP& r, float4 a, float4 b, float4 c, float tbest, float& t, float& b1,
                                float& b2) {
  const float ax = a.x - r.ox, ay = a.y - r.oy, az = a.z - r.oz;
  const float bx = b.x - r.ox, by = b.y - r.oy, bz = b.z - r.oz;
  const float cx = c.x - r.ox, cy = c.y - r.oy, cz = c.z - r.oz;
  const float Akz = pick(ax, ay, az, r.kz), Bkz = pick(bx, by, bz, r.kz), Ckz = pick(cx, cy, cz, r.kz);
  const float Ax = fmaf(-r.Sx, Akz, pick(ax, ay, az, r.kx)), Ay = fmaf(-r.Sy, Akz, pick(ax, ay, az, r.ky));
  const float Bx = fmaf(-r.Sx, Bkz, pick(bx, by, bz, r.kx)), By = fmaf(-r.Sy, Bkz, pick(bx, by, bz, r.ky));
  const float Cx = fmaf(-r.Sx, Ckz, pick(cx, cy, cz, r.kx)), Cy = fmaf(-r.Sy, Ckz, pick(cx, cy, cz, r.ky));
  float U = __fsub_rn(__fmul_rn(Cx, By), __fmul_rn(Cy, Bx));
  float V = __fsub_rn(__fmul_rn(Ax, Cy), __fmul_rn(Ay, Cx));
  float W = __fsub_rn(__fmul_rn(Bx, Ay), __fmul_rn(By, Ax));
  if (U == 0.0f || V == 0.0f || W == 0.0f) {
    U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
    V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
    W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
  }
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

__device__ inline float table_yield(const float* yld, const DevTables& tb, float E, float alpha) {
  float x = (logf(E) - tb.logEmin) * tb.invdlogE;
  x = fminf(fmaxf(x, 0.0f), (float)(tb.nE - 1));
  int i = min((int)floorf(x), tb.nE - 2);
  const float fx = x - (float)i;
  float y = fminf(fmaxf(alpha * tb.thscale, 0.0f), (float)(tb.nth - 1));
  int j = min((int)floorf(y), tb.nth - 2);
  const float fy = y - (float)j;
  const float* row0 = yld + i * tb.nth + j;
  const float* row1 = row0 + tb.nth;
  return (1.0f - fx) * (1.0f - fy) * row0[0] + fx * (1.0f - fy) * row1[0] + (1.0f - fx) * fy * row0[1] +
         fx * fy * row1[1];
}

// piecewise-linear CDF at E
__device__ inline float cdf_at(const float* cE, const float* cF, int n, float E) {
  if (E <= cE[0]) return cF[0];
  if (E >= cE[n - 1]) return cF[n - 1];
  int lo = 0, hi = n - 1;  // cE[lo] <= E < cE[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (cE[mid] <= E)
      lo = mid;
    else
      hi = mid;
  }
  return cF[lo] + (E - cE[lo]) / (cE[lo + 1] - cE[lo]) * (cF[lo + 1] - cF[lo]);
}

// energy where the piecewise-linear CDF first reaches c
__device__ inline float cdf_inv(const float* cE, const float* cF, int n, float c) {
  int lo = 0, hi = n - 1;  // smallest m >= 1 with cF[m] >= c lies in (lo, hi]
  if (!(cF[hi] >= c)) return cE[n - 1];
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (cF[mid] >= c)
      hi = mid;
    else
      lo = mid;
  }
  const int k = hi - 1;
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

__device__ inline int find_job(const DevJob* jobs, int n, uint64_t g) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].gbase <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ inline long long to_fx(float E) { return (long long)llrintf(E * 1048576.0f); }

// ---------------------------------------------------------------- tallies

struct WaveTally {
  unsigned long long* cnt;  // LDS [T_NCOUNT]
  uint32_t* eh;             // LDS [n_ebins]
  uint32_t* ah;             // LDS [n_abins]
};

__device__ inline void tally_cnt(bool mine, const WaveTally& wt, unsigned long long* g, int slot,
                                 unsigned long long v) {
  if (mine)
    atomicAdd(&wt.cnt[slot], v);
  else
    atomicAdd(&g[slot], v);
}

__device__ inline void flush_wave(const WaveTally& wt, unsigned long long* g, int n_eb, int n_ab, uint32_t lane) {
  wave_sync();
  for (int i = lane; i < T_NCOUNT; i += 64) {
    const unsigned long long v = wt.cnt[i];
    if (v) atomicAdd(&g[i], v);
    wt.cnt[i] = 0ull;
  }
  for (int i = lane; i < n_eb; i += 64) {
    const uint32_t v = wt.eh[i];
    if (v) atomicAdd(&g[T_NCOUNT + i], (unsigned long long)v);
    wt.eh[i] = 0u;
  }
  for (int i = lane; i < n_ab; i += 64) {
    const uint32_t v = wt.ah[i];
    if (v) atomicAdd(&g[T_NCOUNT + n_eb + i], (unsigned long long)v);
    wt.ah[i] = 0u;
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
  float te0, te1, te2;  // distances to the x, y, z faces of the cell
  float total;          // path length of earlier segments
  int wraps;
};

__device__ inline void seg_begin(Trav& s, const DevScene& sc) {
  const RayP& r = s.r;
  const float tex = r.dx > 0.0f ? (sc.hi[0] - r.ox) / r.dx : (r.dx < 0.0f ? (sc.lo[0] - r.ox) / r.dx : INFINITY);
  const float tey = r.dy > 0.0f ? (sc.hi[1] - r.oy) / r.dy : (r.dy < 0.0f ? (sc.lo[1] - r.oy) / r.dy : INFINITY);
  const float tez = r.dz > 0.0f ? (sc.hi[2] - r.oz) / r.dz : (r.dz < 0.0f ? (sc.lo[2] - r.oz) / r.dz : INFINITY);
  s.te0 = fmaxf(tex, 0.0f);
  s.te1 = fmaxf(tey, 0.0f);
  s.te2 = fmaxf(tez, 0.0f);
  s.t = fminf(fminf(s.te0, s.te1), s.te2);
  s.idx = -1;
  s.oid = 0x7fffffff;
  s.node = 0;
  s.sp = 0;
}

// One node of the traversal.  Returns true when the segment's traversal has
// finished (stack empty).  The stack keeps its first sd entries in LDS (lstk,
// stride 64 words) and the rest in global memory (gstk, stride 64 words).
__device__ inline bool trav_step(Trav& s, const LaneScene& L, uint32_t* lstk, uint32_t* gstk, int sd, int gd,
                                 uint32_t& visits, uint32_t& tests, bool& ovf) {
  const float4* N = L.nodes + 4 * (size_t)s.node;
  const float4 n0 = N[0], n1 = N[1], n2 = N[2], n3 = N[3];
  ++visits;
  float tl, tr;
  bool hl = box_test(s.r, n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, s.t, tl);
  bool hr = box_test(s.r, n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, s.t, tr);
  const uint32_t cl = __float_as_uint(n3.x), cr = __float_as_uint(n3.y);
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const bool leafhit = side == 0 ? (hl && (cl & kLeafBit)) : (hr && (cr & kLeafBit));
    if (leafhit) {
      const uint32_t k = (side == 0 ? cl : cr) & ~kLeafBit;
      const float4* T = L.tris + 3 * (size_t)k;
      const float4 a = T[0], b = T[1], c = T[2];
      ++tests;
      float t, b1, b2;
      if (tri_test(s.r, a, b, c, s.t, t, b1, b2)) {
        const int32_t oid = (int32_t)__float_as_uint(a.w);
        // closest hit; equal distances go to the lower caller index
        if (t < s.t || (t == s.t && oid < s.oid)) {
          s.t = t;
          s.b1 = b1;
          s.b2 = b2;
          s.idx = (int32_t)k;
          s.oid = oid;
        }
      }
      if (side == 0)
        hl = false;
      else
        hr = false;
    }
  }
  if (hl && hr) {
    const bool lnear = tl <= tr;
    const uint32_t farc = lnear ? cr : cl;
    s.node = lnear ? cl : cr;
    if (s.sp < sd) {
      lstk[s.sp * 64] = farc;
    } else if (s.sp < sd + gd) {
      gstk[(s.sp - sd) * 64] = farc;
    } else {
      ovf = true;
      return true;
    }
    ++s.sp;
    return false;
  }
  if (hl) {
    s.node = cl;
    return false;
  }
  if (hr) {
    s.node = cr;
    return false;
  }
  if (s.sp == 0) return true;
  --s.sp;
  s.node = s.sp < sd ? lstk[s.sp * 64] : gstk[(s.sp - sd) * 64];
  return false;
}

// End of a segment: returns the ray's outcome, or -1 when the ray re-enters
// through the opposite x / y face and traversal continues (section 2.2
// boundaries: periodic in x and y, substrate or open bottom at z_min,
// escape at z_max).
__device__ inline int seg_end(Trav& s, const DevScene& sc, bool ovf, float& px, float& py) {
  if (s.idx >= 0) {
    s.total += s.t;
    return K_HIT;
  }
  const RayP& r = s.r;
  if (s.te2 <= s.te0 && s.te2 <= s.te1) {
    s.total += s.te2;
    if (r.dz > 0.0f) return K_ESCAPE;
    if (sc.flags & 2u) {
      px = r.ox + s.te2 * r.dx;
      py = r.oy + s.te2 * r.dy;
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
  float qx = r.ox + texit * r.dx, qy = r.oy + texit * r.dy, qz = r.oz + texit * r.dz;
  if (s.te0 == texit)
    qx = r.dx > 0.0f ? sc.lo[0] : sc.hi[0];
  else
    qx = fminf(fmaxf(qx, sc.lo[0]), sc.hi[0]);
  if (s.te1 == texit)
    qy = r.dy > 0.0f ? sc.lo[1] : sc.hi[1];
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

// Closest-hit traversal of one generation of rays.  Lanes that finish pick
// up new rays (one atomic per refill of the wave) so that a wave is not held
// by its slowest ray.  MULTI: rays may belong to different jobs.
template <bool MULTI>
__global__ __launch_bounds__(256) void k_traverse(TraverseArgs a) {
  const int wpb = blockDim.x >> 6;
  const int w = threadIdx.x >> 6;
  const uint32_t lane = lane_id();
  const uint64_t lt = (1ull << lane) - 1ull;
  uint32_t* lstk = reinterpret_cast<uint32_t*>(smem) + (size_t)w * a.lds_stack * 64 + lane;
  uint32_t* gstk = a.gstack + ((size_t)(blockIdx.x * wpb + w) * a.gstack_depth) * 64 + lane;
  const uint32_t count = a.src == 1 ? min(*a.count_in, a.qcap) : a.count;

  Trav s;
  LaneScene L;
  int job = 0;
  uint32_t item = 0, visits = 0, tests = 0;
  bool have = false, ovf = false;
  bool exhausted = false;
  if (!MULTI) {
    L.nodes = a.jobs[0].sc.nodes;
    L.tris = a.jobs[0].sc.tris;
    L.n_tris = a.jobs[0].sc.n_tris;
    L.flags = a.jobs[0].sc.flags;
  }
  for (;;) {
    const uint64_t idle = __ballot(!have);
    const uint32_t nidle = (uint32_t)__popcll(idle);
    if (!exhausted && nidle >= (uint32_t)a.refill) {
      uint32_t base = 0;
      if (lane == 0) base = atomicAdd(a.work, nidle);
      base = __shfl(base, 0, 64);
      if (base + nidle >= count) exhausted = true;
      if (!have) {
        item = base + (uint32_t)__popcll(idle & lt);
        if (item < count) {
          float ox, oy, oz, dx, dy, dz;
          if (a.src == 0) {
            const uint64_t g = a.chunk_lo + item;
            job = MULTI ? find_job(a.jobs, a.n_jobs, g) : 0;
            primary_ray(a.jobs[job], g, ox, oy, oz, dx, dy, dz);
          } else if (a.src == 1) {
            ox = a.qin.ox[item];
            oy = a.qin.oy[item];
            oz = a.qin.oz[item];
            dx = a.qin.dx[item];
            dy = a.qin.dy[item];
            dz = a.qin.dz[item];
            if (MULTI) job = (int)(a.qin.meta[item] >> 4);
          } else {
            const float* q = a.rays + 6 * (size_t)item;
            ox = q[0];
            oy = q[1];
            oz = q[2];
            dx = q[3];
            dy = q[4];
            dz = q[5];
          }
          if (MULTI) {
            L.nodes = a.jobs[job].sc.nodes;
            L.tris = a.jobs[job].sc.tris;
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
          seg_begin(s, a.jobs[job].sc);
          have = true;
        }
      }
    }
    if (__ballot(have) == 0ull) {
      if (exhausted) break;
      continue;
    }
    if (have) {
      bool done = L.n_tris == 0 || trav_step(s, L, lstk, gstk, a.lds_stack, a.gstack_depth, visits, tests, ovf);
      if (done) {
        float px = 0.f, py = 0.f;
        const DevScene& sc = a.jobs[job].sc;
        const int kind = seg_end(s, sc, ovf, px, py);
        if (kind < 0) {
          seg_begin(s, sc);
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
          a.hit.code[item] = code;
          a.hit.f0[item] = f0;
          a.hit.f1[item] = f1;
          a.hit.t[item] = s.total;
          a.hit.visits[item] = visits;
          a.hit.tests[item] = tests;
          a.hit.wraps[item] = (uint32_t)s.wraps | (ovf ? 0x80000000u : 0u);
          if (ovf) atomicOr(a.err, 2u);
          have = false;
        }
      }
    }
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
// with one atomic per wave.  Tables sit in LDS; tallies in per-wave LDS
// blocks tagged with the job they belong to.
__global__ __launch_bounds__(256) void k_shade(ShadeArgs a) {
  const int wpb = blockDim.x >> 6;
  const int w = threadIdx.x >> 6;
  const uint32_t lane = lane_id();
  const DevTables& tb = a.tb;
  const int nY = tb.nE * tb.nth;
  float* s_yld = reinterpret_cast<float*>(smem);
  float* s_cE = s_yld + nY;
  float* s_cF = s_cE + tb.ncdf;
  size_t off = ((size_t)(nY + 2 * tb.ncdf) * 4 + 15) & ~(size_t)15;
  unsigned long long* s_cnt = reinterpret_cast<unsigned long long*>(smem + off);
  off += (size_t)wpb * T_NCOUNT * 8;
  uint32_t* s_eh = reinterpret_cast<uint32_t*>(smem + off);
  off += (size_t)wpb * a.n_ebins * 4;
  uint32_t* s_ah = reinterpret_cast<uint32_t*>(smem + off);

  const uint32_t count = a.gen == 0 ? a.n_gen0 : min(*a.count_in, a.qcap);
  if ((uint32_t)blockIdx.x * blockDim.x >= count) return;  // whole workgroup idle
  for (int i = threadIdx.x; i < nY; i += blockDim.x) s_yld[i] = tb.yld[i];
  for (int i = threadIdx.x; i < tb.ncdf; i += blockDim.x) {
    s_cE[i] = tb.cdfE[i];
    s_cF[i] = tb.cdfF[i];
  }
  for (int i = threadIdx.x; i < wpb * T_NCOUNT; i += blockDim.x) s_cnt[i] = 0ull;
  for (int i = threadIdx.x; i < wpb * a.n_ebins; i += blockDim.x) s_eh[i] = 0u;
  for (int i = threadIdx.x; i < wpb * a.n_abins; i += blockDim.x) s_ah[i] = 0u;
  __syncthreads();

  WaveTally wt{s_cnt + w * T_NCOUNT, s_eh + w * a.n_ebins, s_ah + w * a.n_abins};
  int tag = -1;
  const uint32_t stride = gridDim.x * (uint32_t)blockDim.x;
  for (uint32_t base = (blockIdx.x * wpb + w) * 64u; base < count; base += stride) {
    const uint32_t item = base + lane;
    const bool active = item < count;

    float ox = 0.f, oy = 0.f, oz = 0.f, dx = 0.f, dy = 0.f, dz = -1.f, E = 0.f;
    uint32_t path = 0, ci = 0;
    int gen = a.gen, job = 0;
    if (active) {
      if (a.gen == 0) {
        const uint64_t g = a.chunk_lo + item;
        job = find_job(a.jobs, a.n_jobs, g);
        primary_ray(a.jobs[job], g, ox, oy, oz, dx, dy, dz);
        E = a.jobs[job].E0;
        ci = item;
      } else {
        dx = a.qin.dx[item];
        dy = a.qin.dy[item];
        dz = a.qin.dz[item];
        E = a.qin.E[item];
        path = a.qin.path[item];
        ci = a.qin.ci[item];
        const uint32_t m = a.qin.meta[item];
        gen = (int)(m & 15u);
        job = (int)(m >> 4);
      }
    }
    (void)ox;
    (void)oy;
    (void)oz;
    const int j0 = __shfl(job, 0, 64);
    if (j0 != tag) {
      if (tag >= 0) flush_wave(wt, a.jobs[tag].tally, a.n_ebins, a.n_abins, lane);
      tag = j0;
    }
    const DevJob& J = a.jobs[job];
    const bool mine = job == tag;
    unsigned long long* gt = J.tally;

    int nd = 0;
    float px = 0.f, py = 0.f, pz = 0.f, nx = 0.f, ny = 0.f, nz = 1.f;
    if (active) {
      const int32_t code = a.hit.code[item];
      const float f0 = a.hit.f0[item], f1 = a.hit.f1[item];
      const uint32_t wr = a.hit.wraps[item];
      tally_cnt(mine, wt, gt, T_RAYS, 1ull);
      tally_cnt(mine, wt, gt, T_VISITS, a.hit.visits[item]);
      tally_cnt(mine, wt, gt, T_TESTS, a.hit.tests[item]);
      if (wr & 0x7fffffffu) tally_cnt(mine, wt, gt, T_WRAPS, (unsigned long long)(wr & 0x7fffffffu));
      if (wr & 0x80000000u) tally_cnt(mine, wt, gt, T_STACKOVF, 1ull);
      if (code == -1) {
        tally_cnt(mine, wt, gt, T_ESCAPED, 1ull);
        tally_cnt(mine, wt, gt, T_E_ESC_FX, (unsigned long long)to_fx(E));
        int eb = (int)floorf(E / J.E0 * (float)a.n_ebins);
        eb = min(max(eb, 0), a.n_ebins - 1);
        const float pol = acosf(fminf(dz, 1.0f)) * kDeg;
        int ab = (int)floorf(pol * (1.0f / 90.0f) * (float)a.n_abins);
        ab = min(max(ab, 0), a.n_abins - 1);
        if (mine) {
          atomicAdd(&wt.eh[eb], 1u);
          atomicAdd(&wt.ah[ab], 1u);
        } else {
          atomicAdd(&gt[T_NCOUNT + eb], 1ull);
          atomicAdd(&gt[T_NCOUNT + a.n_ebins + ab], 1ull);
        }
        atomicAdd(&a.ppc[ci], 1u);
      } else if (code == -3) {
        tally_cnt(mine, wt, gt, T_LOST, 1ull);
        tally_cnt(mine, wt, gt, T_E_DEP_FX, (unsigned long long)to_fx(E));
      } else {
        if (code == -2) {
          tally_cnt(mine, wt, gt, T_SUBSTRATE, 1ull);
          px = f0;
          py = f1;
          pz = J.sc.lo[2];
        } else {
          const float4* T = J.sc.tris + 3 * (size_t)code;
          const float4 v0 = T[0], v1 = T[1], v2 = T[2];
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
        if (gen >= a.max_gen) {
          tally_cnt(mine, wt, gt, T_TRUNCATED, 1ull);
          tally_cnt(mine, wt, gt, T_E_DEP_FX, (unsigned long long)to_fx(E));
        } else {
          tally_cnt(mine, wt, gt, T_ABSORBED, 1ull);
          if (E <= tb.Ec) {
            tally_cnt(mine, wt, gt, T_E_DEP_FX, (unsigned long long)to_fx(E));
          } else {
            const float cosa = fminf(fmaxf(-(dx * nx + dy * ny + dz * nz), 0.0f), 1.0f);
            const float alpha = acosf(cosa) * kDeg;
            const float delta = table_yield(s_yld, tb, E, alpha);
            const uint64_t pid = J.pid0 + (a.chunk_lo + ci - J.gbase);
            const U4 u = philox(J.seed, (uint32_t)pid, (uint32_t)(pid >> 32), path, 1u);
            const float fl = floorf(delta);
            nd = (int)fl + (u01(u.x) < delta - fl ? 1 : 0);
            if (nd == 0) tally_cnt(mine, wt, gt, T_E_DEP_FX, (unsigned long long)to_fx(E));
          }
        }
      }
    }

    // ---- daughters: one queue reservation per wave
    const uint32_t incl = wave_incl_scan((uint32_t)nd, lane);
    const uint32_t total = __shfl(incl, 63, 64);
    if (total == 0u) continue;
    uint32_t obase = 0;
    if (lane == 0) obase = atomicAdd(a.count_out, total);
    obase = __shfl(obase, 0, 64);
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
      for (int d = 0; d < nd; ++d) {
        const U4 u = philox(J.seed, (uint32_t)pid, (uint32_t)(pid >> 32), path, 2u + (uint32_t)d);
        float Ed = cdf_inv(s_cE, s_cF, tb.ncdf, u01(u.x) * cdf_at(s_cE, s_cF, tb.ncdf, Eav));
        Ed = fminf(Ed, Eav);
        Eav -= Ed;
        fx_left -= to_fx(Ed);
        const float xb = u01(u.y);
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
          a.qout.ox[slot] = qx;
          a.qout.oy[slot] = qy;
          a.qout.oz[slot] = qz;
          a.qout.dx[slot] = ddx;
          a.qout.dy[slot] = ddy;
          a.qout.dz[slot] = ddz;
          a.qout.E[slot] = Ed;
          a.qout.path[slot] = path * 8u + (uint32_t)d + 1u;
          a.qout.ci[slot] = ci;
          a.qout.meta[slot] = (uint32_t)(gen + 1) | ((uint32_t)job << 4);
        } else {
          ++dropped;
        }
      }
      tally_cnt(mine, wt, gt, T_E_DEP_FX, (unsigned long long)fx_left);
      tally_cnt(mine, wt, gt, T_SPAWNED, (unsigned long long)nd);
      if (dropped) {
        tally_cnt(mine, wt, gt, T_DROPPED, dropped);
        atomicOr(a.err, 1u);
      }
    }
  }
  if (tag >= 0) flush_wave(wt, a.jobs[tag].tally, a.n_ebins, a.n_abins, lane);
}

__global__ void k_chunk_reduce(const DevJob* jobs, int32_t n_jobs, const uint32_t* __restrict__ ppc, uint32_t n,
                               uint64_t chunk_lo) {
  const uint32_t lane = lane_id();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t start = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t iters = (n + stride - 1) / stride;
  for (uint64_t it = 0; it < iters; ++it) {
    const uint64_t i = start + it * stride;
    const bool valid = i < n;
    int job = 0;
    unsigned long long c2 = 0;
    if (valid) {
      const uint64_t g = chunk_lo + i;
      job = find_job(jobs, n_jobs, g);
      const uint32_t c = ppc[i];
      c2 = (unsigned long long)c * c;
      if (jobs[job].pp_escaped) jobs[job].pp_escaped[g - jobs[job].gbase] = c;
    }
    const int j0 = __shfl(job, 0, 64);
    const bool uniform = __all(!valid || job == j0);
    if (uniform) {
      unsigned long long s = c2;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0 && s) atomicAdd(&jobs[j0].tally[T_C2], s);
    } else if (valid && c2) {
      atomicAdd(&jobs[job].tally[T_C2], c2);
    }
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
typedef float f4v __attribute__((ext_vector_type(4)));

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

size_t traverse_lds_bytes(int lds_stack, int block) { return (size_t)(block / 64) * lds_stack * 64 * 4; }

size_t shade_lds_bytes(const DevTables& tb, int n_ebins, int n_abins, int block) {
  const int wpb = block / 64;
  size_t off = ((size_t)(tb.nE * tb.nth + 2 * tb.ncdf) * 4 + 15) & ~(size_t)15;
  off += (size_t)wpb * T_NCOUNT * 8;
  off += (size_t)wpb * n_ebins * 4;
  off += (size_t)wpb * n_abins * 4;
  return off;
}

hipError_t launch_traverse(const TraverseArgs& a, bool multi, int grid, int block, hipStream_t s) {
  const size_t lds = traverse_lds_bytes(a.lds_stack, block);
  if (multi)
    k_traverse<true><<<grid, block, lds, s>>>(a);
  else
    k_traverse<false><<<grid, block, lds, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_shade(const ShadeArgs& a, int grid, int block, hipStream_t s) {
  const size_t lds = shade_lds_bytes(a.tb, a.n_ebins, a.n_abins, block);
  k_shade<<<grid, block, lds, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_hit_ids(const float4* tris, const int32_t* code, int64_t n, int32_t* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_hit_ids<<<(int)((n + 255) / 256), 256, 0, s>>>(tris, code, n, out);
  return hipGetLastError();
}

hipError_t launch_chunk_reduce(const DevJob* jobs, int32_t n_jobs, const uint32_t* ppc, uint32_t n,
                               uint64_t chunk_lo, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int grid = (int)((n + 255) / 256);
  if (grid > 4096) grid = 4096;
  k_chunk_reduce<<<grid, 256, 0, s>>>(jobs, n_jobs, ppc, n, chunk_lo);
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
