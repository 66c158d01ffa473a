// Shading on gfx950 (section 2.2), one lane per ray: k_shade turns the
// traversal's hit records into outcomes and daughters.  The local incidence
// angle and the flat-surface tables give the daughter count (stochastic
// rounding, footnote of section 2.2), energies (inverse of the tabulated CDF
// truncated to the energy still available) and cosine-law directions;
// daughters are appended to the next queue with one atomic per workgroup step;
// tallies accumulate per lane and per job.  Random numbers: Philox4x32-10
// keyed by the job seed, counter (primary id, 0, path code, draw); draw 0 =
// birth of a primary, 1 = daughter count, 2 + d = daughter d; a daughter's
// path code is parent * 8 + d + 1.
#include "device_util.h"
#include "shade_kernels.h"

namespace rtmc {
namespace {

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

extern __shared__ __align__(16) unsigned char smem[];

// Where a ray ended on a surface: the hit point and the unit normal of the
// element (triangle, or the substrate plane at z_min with normal +z).
__device__ inline void hit_frame(const DevJob& J, int32_t code, float f0, float f1, float& px, float& py, float& pz,
                                 float& nx, float& ny, float& nz) {
  if (code == -2) {
    px = f0;
    py = f1;
    pz = J.sc.lo[2];
    nx = 0.f;
    ny = 0.f;
    nz = 1.f;
    return;
  }
  // the vertices from the triangle's 64-byte rotated record (x y z x y per
  // vertex, then the caller's index): one aligned line segment per gather,
  // where the 48-byte sorted record straddles two lines three times in eight
  const GAS f4v* R = (const GAS f4v*)J.sc.tris_t + 4 * (size_t)code;
  const f4v r0 = R[0], r1 = R[1], r2 = R[2], r3 = R[3];
  const f4v v0 = {r0.x, r0.y, r0.z, 0.f}, v1 = {r1.y, r1.z, r1.w, 0.f}, v2 = {r2.z, r2.w, r3.x, 0.f};
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

// Local incidence angle in degrees: the angle between the reversed ray and
// the element normal, arccos(-d . n) in [0, 90].
__device__ inline float incidence_deg(float dx, float dy, float dz, float nx, float ny, float nz) {
  return acosf(fminf(fmaxf(-(dx * nx + dy * ny + dz * nz), 0.0f), 1.0f)) * kDeg;
}

// Table views of one shading workgroup (yield grid and CDF in LDS).
struct ShadeTabs {
  const LAS float* yld;
  const LAS float* cE;
  const LAS float* cF;
  const LAS uint16_t* gF;
  const LAS uint16_t* gE;
};

// The nd daughters of one emitting hit (section 2.2): energies from the
// spectrum truncated to what the parent still has (or the paper's rule),
// cosine-law directions about the normal, spawned just off the surface,
// written to slots first .. first + nd - 1 of the next queue.
__device__ inline void spawn(const ShadeArgs& a, const ShadeTabs& st, const DevJob& J, int job, int gen, float E,
                             uint32_t path, uint32_t ci, float px, float py, float pz, float nx, float ny, float nz,
                             float es, int nd, uint32_t first, bool mine, WaveTally& wt, const JobTab* jt) {
  const DevTables& tb = a.tb;
  unsigned long long* gt = J.tally;
  const uint64_t pid = J.pid0 + (a.chunk_lo + ci - J.gbase);
  float Eav = E;
  long long fx_left = to_fx(E);
  float3 t1, t2;
  onb(nx, ny, nz, t1, t2);
  const float Lx = J.sc.hi[0] - J.sc.lo[0], Ly = J.sc.hi[1] - J.sc.lo[1];
  const bool periodic = (J.sc.flags & 1u) != 0;
  const bool paper = tb.emission == kEmitPaper;
  uint32_t dropped = 0;
  float xi_pair = 0.0f;
  for (int d = 0; d < nd; ++d) {
    const U4 u = philox(J.seed, (uint32_t)pid, (uint32_t)(pid >> 32), path, 2u + (uint32_t)d);
    float Ed, xb;  // energy and sin^2 of the angle from the normal
    if (!paper) {
      Ed = cdf_inv(st.cE, st.cF, tb.ncdf, st.gF,
                   u01(u.x) * cdf_at(st.cE, st.cF, tb.ncdf, st.gE, tb.e1bits, tb.eshift, Eav));
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
    // azimuth 2 pi xi: sine and cosine of pi (2 xi), 2 xi exact in FP32
    float sp, cp;
    sincospif(2.0f * u01(u.z), &sp, &cp);
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
  const ShadeTabs st{s_yld, s_cE, s_cF, s_gF, s_gE};

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

    float dx = 0.f, dy = 0.f, dz = -1.f, E = 0.f;
    uint32_t path = 0, ci = 0;
    int gen = a.gen, job = 0;
    if (active) {
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
    float px = 0.f, py = 0.f, pz = 0.f, nx = 0.f, ny = 0.f, nz = 1.f, es = 0.f;
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
        if (code == -2) tally_cnt(mine, wt, gt, T_SUBSTRATE, 1ull, jt, job);
        // the hit point and normal only where they are used: a hit that may
        // emit (above E_c, below the last generation), or the depth histogram
        // (most daughters arrive below E_c and need no triangle gather)
        if (a.n_zbins > 0 || (gen < a.max_gen && E > tb.Ec)) hit_frame(J, code, f0, f1, px, py, pz, nx, ny, nz);
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
            const float alpha = incidence_deg(dx, dy, dz, nx, ny, nz);
            const float delta = table_yield(s_yld, tb, E, alpha);
            const uint64_t pid = J.pid0 + (a.chunk_lo + ci - J.gbase);
            const U4 u = philox(J.seed, (uint32_t)pid, (uint32_t)(pid >> 32), path, 1u);
            const float fl = floorf(delta);
            nd = (int)fl + (u01(u.x) < delta - fl ? 1 : 0);
            if (nd == 0) tally_cnt(mine, wt, gt, T_E_DEP_FX, (unsigned long long)to_fx(E), jt, job);
            // the paper's rule: E_SEE at (E, alpha)
            if (nd > 0 && tb.emission == kEmitPaper) es = table_yield((const GAS float*)tb.esee, tb, E, alpha);
          }
        }
      }
    }

    // ---- one queue reservation per workgroup step
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
    if (nd > 0)
      spawn(a, st, J, job, gen, E, path, ci, px, py, pz, nx, ny, nz, es, nd, s_wbase[w] + incl - (uint32_t)nd, mine,
            wt, jt);
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

__global__ void k_copy_rays(RayQueue q, const uint32_t* count, uint32_t qcap, float* out, uint32_t n_max,
                            uint32_t* n_out) {
  const uint32_t n = min(min(*count, qcap), n_max);
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_out = n;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    float* r = out + 6 * (size_t)i;
    r[0] = q.ox[i];
    r[1] = q.oy[i];
    r[2] = q.oz[i];
    r[3] = q.dx[i];
    r[4] = q.dy[i];
    r[5] = q.dz[i];
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

size_t shade_lds_bytes(const DevTables& tb, int n_hist, int block, int n_jobs) {
  const int wpb = block / 64;
  size_t off = ((size_t)(tb.nE * tb.nth + 2 * tb.ncdf) * 4 + 4 * kGuide + 15) & ~(size_t)15;
  const size_t per_wave = (size_t)wpb * n_hist * 4;
  const size_t per_job = n_jobs <= kShadeJobs
                             ? (size_t)n_jobs * ((T_NCOUNT * 8 + n_hist * 4 + 7) & ~7)
                             : 0;
  return off + (per_wave > per_job ? per_wave : per_job);
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

hipError_t launch_chunk_reduce(const DevJob* jobs, int32_t j_lo, int32_t j_hi, const uint32_t* ppc, uint32_t n,
                               uint64_t chunk_lo, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int grid = (int)((n + 255) / 256);
  if (grid > 1024) grid = 1024;
  k_chunk_reduce<<<grid, 256, 0, s>>>(jobs, j_lo, j_hi, ppc, n, chunk_lo);
  return hipGetLastError();
}

hipError_t launch_copy_rays(const RayQueue& q, const uint32_t* count, uint32_t qcap, float* out, uint32_t n_max,
                            uint32_t* n_out, hipStream_t s) {
  k_copy_rays<<<1024, 256, 0, s>>>(q, count, qcap, out, n_max, n_out);
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
