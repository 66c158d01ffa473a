// Ray tracing Monte Carlo on gfx950: one lane per ray.
//
// One launch processes one generation of rays (the paper's tree of branches,
// section 2.2, handled breadth-first across all primaries): generation 0 is
// generated from primary ids, later generations are read from the daughter
// queue the previous launch filled.  Per ray:
//   - closest front-facing triangle by BVH traversal (section 2.1): robust
//     slab tests against both child boxes of a 64-byte node record, and the
//     watertight ray/triangle test of Woop, Benthin and Wald (JCGT 2013) with
//     back-face culling; periodic re-entry through the x / y faces, escape
//     through z_max, the substrate plane at z_min (section 2.2);
//   - on a hit, the local incidence angle and the flat-surface tables give the
//     daughter count (stochastic rounding, footnote of section 2.2), energies
//     (inverse of the tabulated CDF, truncated to the energy still available)
//     and cosine-law directions;
//   - daughters are appended to the next queue with one atomic per wave
//     (wave prefix sum of the per-lane counts);
//   - tallies go to per-wave LDS counters and histograms, flushed to the
//     job's global tally block once per wave.
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the job seed,
// counter (primary id, 0, path code, draw); draw 0 = birth of a primary,
// 1 = daughter count, 2 + d = daughter d; a daughter's path code is
// parent * 8 + d + 1.
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

struct Hit {
  float t, b1, b2;
  int32_t idx;  // sorted triangle index, -1 none
  int32_t oid;  // caller's triangle index
};

// Closest hit with 0 < t <= tmax.  The stack keeps its first sd entries in
// LDS (lstk, stride 64 words) and the rest in global memory (gstk, stride 64).
__device__ inline void traverse(const RayP& r, const float4* __restrict__ nodes, const float4* __restrict__ tris,
                                float tmax, Hit& h, uint32_t* lstk, uint32_t* gstk, int sd, int gd, uint32_t& visits,
                                uint32_t& tests, bool& ovf) {
  h.t = tmax;
  h.idx = -1;
  h.oid = 0x7fffffff;
  uint32_t node = 0;
  int sp = 0;
  for (;;) {
    const float4* N = nodes + 4 * (size_t)node;
    const float4 n0 = N[0], n1 = N[1], n2 = N[2], n3 = N[3];
    ++visits;
    float tl, tr;
    bool hl = box_test(r, n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, h.t, tl);
    bool hr = box_test(r, n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, h.t, tr);
    const uint32_t cl = __float_as_uint(n3.x), cr = __float_as_uint(n3.y);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const bool leafhit = side == 0 ? (hl && (cl & kLeafBit)) : (hr && (cr & kLeafBit));
      if (leafhit) {
        const uint32_t k = (side == 0 ? cl : cr) & ~kLeafBit;
        const float4* T = tris + 3 * (size_t)k;
        const float4 a = T[0], b = T[1], c = T[2];
        ++tests;
        float t, b1, b2;
        if (tri_test(r, a, b, c, h.t, t, b1, b2)) {
          const int32_t oid = (int32_t)__float_as_uint(a.w);
          if (t < h.t || (t == h.t && oid < h.oid)) {
            h.t = t;
            h.b1 = b1;
            h.b2 = b2;
            h.idx = (int32_t)k;
            h.oid = oid;
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
      node = lnear ? cl : cr;
      if (sp < sd) {
        lstk[sp * 64] = farc;
      } else if (sp < sd + gd) {
        gstk[(sp - sd) * 64] = farc;
      } else {
        ovf = true;
        return;
      }
      ++sp;
    } else if (hl) {
      node = cl;
    } else if (hr) {
      node = cr;
    } else {
      if (sp == 0) return;
      --sp;
      node = sp < sd ? lstk[sp * 64] : gstk[(sp - sd) * 64];
    }
  }
}

enum { K_HIT = 0, K_ESCAPE = 1, K_SUBSTRATE = 2, K_LOST = 3 };

struct PathOut {
  int kind;
  Hit h;
  float px, py, pz;  // substrate point
  float t_total;
  int wraps;
};

// Follow one ray through the periodic cell (section 2.2 boundaries).
__device__ inline void trace_path(const DevScene& sc, float ox, float oy, float oz, float dx, float dy, float dz,
                                  uint32_t* lstk, uint32_t* gstk, int sd, int gd, uint32_t& visits,
                                  uint32_t& tests, bool& ovf, PathOut& out) {
  RayP r;
  ray_setup(r, dx, dy, dz);
  float total = 0.0f;
  int wraps = 0;
  const bool periodic = (sc.flags & 1u) != 0;
  for (;;) {
    const float tex = dx > 0.0f ? (sc.hi[0] - ox) / dx : (dx < 0.0f ? (sc.lo[0] - ox) / dx : INFINITY);
    const float tey = dy > 0.0f ? (sc.hi[1] - oy) / dy : (dy < 0.0f ? (sc.lo[1] - oy) / dy : INFINITY);
    const float tez = dz > 0.0f ? (sc.hi[2] - oz) / dz : (dz < 0.0f ? (sc.lo[2] - oz) / dz : INFINITY);
    const float te0 = fmaxf(tex, 0.0f), te1 = fmaxf(tey, 0.0f), te2 = fmaxf(tez, 0.0f);
    const float texit = fminf(fminf(te0, te1), te2);
    r.ox = ox;
    r.oy = oy;
    r.oz = oz;
    Hit h;
    h.idx = -1;
    if (sc.n_tris > 0) traverse(r, sc.nodes, sc.tris, texit, h, lstk, gstk, sd, gd, visits, tests, ovf);
    if (h.idx >= 0) {
      out.kind = K_HIT;
      out.h = h;
      out.t_total = total + h.t;
      out.wraps = wraps;
      return;
    }
    if (te2 <= te0 && te2 <= te1) {
      out.t_total = total + te2;
      out.wraps = wraps;
      if (dz > 0.0f) {
        out.kind = K_ESCAPE;
      } else if (sc.flags & 2u) {
        out.kind = K_SUBSTRATE;
        out.px = ox + te2 * dx;
        out.py = oy + te2 * dy;
        out.pz = sc.lo[2];
      } else {
        out.kind = K_LOST;
      }
      return;
    }
    if (!periodic || ovf) {
      out.kind = K_LOST;
      out.t_total = total + texit;
      out.wraps = wraps;
      return;
    }
    total += texit;
    float px = ox + texit * dx, py = oy + texit * dy, pz = oz + texit * dz;
    if (te0 == texit)
      px = dx > 0.0f ? sc.lo[0] : sc.hi[0];
    else
      px = fminf(fmaxf(px, sc.lo[0]), sc.hi[0]);
    if (te1 == texit)
      py = dy > 0.0f ? sc.lo[1] : sc.hi[1];
    else
      py = fminf(fmaxf(py, sc.lo[1]), sc.hi[1]);
    pz = fminf(fmaxf(pz, sc.lo[2]), sc.hi[2]);
    ox = px;
    oy = py;
    oz = pz;
    if (++wraps > kWrapMax) {
      out.kind = K_LOST;
      out.t_total = total;
      out.wraps = wraps;
      return;
    }
  }
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

extern __shared__ __align__(16) unsigned char smem[];

__global__ __launch_bounds__(1024) void k_trace(TraceArgs a) {
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
  off += (size_t)wpb * a.n_abins * 4;
  off = (off + 15) & ~(size_t)15;
  uint32_t* s_stk = reinterpret_cast<uint32_t*>(smem + off);

  for (int i = threadIdx.x; i < nY; i += blockDim.x) s_yld[i] = tb.yld[i];
  for (int i = threadIdx.x; i < tb.ncdf; i += blockDim.x) {
    s_cE[i] = tb.cdfE[i];
    s_cF[i] = tb.cdfF[i];
  }
  for (int i = threadIdx.x; i < wpb * T_NCOUNT; i += blockDim.x) s_cnt[i] = 0ull;
  for (int i = threadIdx.x; i < wpb * a.n_ebins; i += blockDim.x) s_eh[i] = 0u;
  for (int i = threadIdx.x; i < wpb * a.n_abins; i += blockDim.x) s_ah[i] = 0u;
  __syncthreads();

  // the counter can run past the capacity when appends overflow: never read beyond it
  const uint32_t count = a.gen == 0 ? a.n_gen0 : min(*a.count_in, a.qcap);
  WaveTally wt{s_cnt + w * T_NCOUNT, s_eh + w * a.n_ebins, s_ah + w * a.n_abins};
  uint32_t* lstk = s_stk + (size_t)w * a.lds_stack * 64 + lane;
  uint32_t* gstk = a.gstack + ((size_t)(blockIdx.x * wpb + w) * a.gstack_depth) * 64 + lane;
  int tag = -1;

  for (;;) {
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(a.work, 64u);
    base = __shfl(base, 0, 64);
    if (base >= count) break;
    const uint32_t item = base + lane;
    const bool active = item < count;

    float ox = 0.f, oy = 0.f, oz = 0.f, dx = 0.f, dy = 0.f, dz = -1.f, E = 0.f;
    uint32_t path = 0, ci = 0;
    int gen = a.gen, job = 0;
    if (active) {
      if (a.gen == 0) {
        const uint64_t g = a.chunk_lo + item;
        job = find_job(a.jobs, a.n_jobs, g);
        const DevJob& J = a.jobs[job];
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
        E = J.E0;
        ci = item;
      } else {
        ox = a.qin.ox[item];
        oy = a.qin.oy[item];
        oz = a.qin.oz[item];
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
      uint32_t visits = 0, tests = 0;
      bool ovf = false;
      PathOut po;
      trace_path(J.sc, ox, oy, oz, dx, dy, dz, lstk, gstk, a.lds_stack, a.gstack_depth, visits, tests, ovf, po);
      tally_cnt(mine, wt, gt, T_RAYS, 1ull);
      tally_cnt(mine, wt, gt, T_VISITS, visits);
      tally_cnt(mine, wt, gt, T_TESTS, tests);
      if (po.wraps) tally_cnt(mine, wt, gt, T_WRAPS, (unsigned long long)po.wraps);
      if (ovf) {
        tally_cnt(mine, wt, gt, T_STACKOVF, 1ull);
        atomicOr(a.err, 2u);
      }
      if (po.kind == K_ESCAPE) {
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
      } else if (po.kind == K_LOST) {
        tally_cnt(mine, wt, gt, T_LOST, 1ull);
        tally_cnt(mine, wt, gt, T_E_DEP_FX, (unsigned long long)to_fx(E));
      } else {
        if (po.kind == K_SUBSTRATE) {
          tally_cnt(mine, wt, gt, T_SUBSTRATE, 1ull);
          px = po.px;
          py = po.py;
          pz = po.pz;
        } else {
          const float4* T = J.sc.tris + 3 * (size_t)po.h.idx;
          const float4 v0 = T[0], v1 = T[1], v2 = T[2];
          const float b1 = po.h.b1, b2 = po.h.b2, b0 = 1.0f - b1 - b2;
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

// First surface reached by each ray (parity entry point).
__global__ __launch_bounds__(1024) void k_first_hit(DevScene sc, const float* __restrict__ rays, int64_t n,
                                                    int32_t* __restrict__ tri_out, float* __restrict__ t_out,
                                                    uint32_t* gstack, int sd, int gd) {
  const int wpb = blockDim.x >> 6;
  const int w = threadIdx.x >> 6;
  const uint32_t lane = lane_id();
  uint32_t* s_stk = reinterpret_cast<uint32_t*>(smem);
  uint32_t* lstk = s_stk + (size_t)w * sd * 64 + lane;
  uint32_t* gstk = gstack + ((size_t)(blockIdx.x * wpb + w) * gd) * 64 + lane;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // every lane of a wave runs the same number of iterations
  const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t iters = (n + stride - 1) / stride;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t i = start + it * stride;
    if (i >= n) continue;
    const float* r = rays + 6 * i;
    uint32_t visits = 0, tests = 0;
    bool ovf = false;
    PathOut po;
    trace_path(sc, r[0], r[1], r[2], r[3], r[4], r[5], lstk, gstk, sd, gd, visits, tests, ovf, po);
    int32_t id;
    if (po.kind == K_HIT)
      id = po.h.oid;
    else if (po.kind == K_ESCAPE)
      id = -1;
    else if (po.kind == K_SUBSTRATE)
      id = -2;
    else
      id = -3;
    tri_out[i] = id;
    t_out[i] = po.t_total;
  }
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

size_t trace_lds_bytes(const TraceArgs& a, int block) {
  const int wpb = block / 64;
  size_t off = ((size_t)(a.tb.nE * a.tb.nth + 2 * a.tb.ncdf) * 4 + 15) & ~(size_t)15;
  off += (size_t)wpb * T_NCOUNT * 8;
  off += (size_t)wpb * a.n_ebins * 4;
  off += (size_t)wpb * a.n_abins * 4;
  off = (off + 15) & ~(size_t)15;
  off += (size_t)wpb * a.lds_stack * 64 * 4;
  return off;
}

hipError_t launch_trace(const TraceArgs& a, int grid, int block, hipStream_t s) {
  const size_t lds = trace_lds_bytes(a, block);
  k_trace<<<grid, block, lds, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_first_hit(DevScene sc, const float* rays, int64_t n, int32_t* tri_out, float* t_out,
                            uint32_t* gstack, int lds_stack, int gstack_depth, int grid, int block, hipStream_t s) {
  const size_t lds = (size_t)(block / 64) * lds_stack * 64 * 4;
  k_first_hit<<<grid, block, lds, s>>>(sc, rays, n, tri_out, t_out, gstack, lds_stack, gstack_depth);
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
