// Closest-hit traversal on gfx950 (section 2.1), one lane per ray.
//
// A generation of rays (the paper's tree of branches, section 2.2, handled
// breadth-first across all primaries) is processed by two launches, this
// file's k_traverse and shade.hip's k_shade:
//   k_traverse: closest front-facing triangle by BVH traversal (section 2.1):
//     conservative slab tests against the four byte-quantized child boxes of
//     a 64-byte node and the watertight ray/triangle test of Woop, Benthin and
//     Wald (JCGT 2013) with back-face culling; periodic re-entry through the
//     x / y faces, escape through z_max, substrate plane at z_min (section
//     2.2).  Persistent waves whose lanes refill from the generation's queue
//     once enough of them are done.  Output: one 28-byte hit record per ray.
// Generation 0 is written to the queue from primary ids by k_primaries, so
// both launches read it like any other generation (draw 0 of a primary's
// Philox stream gives its origin, azimuth and, for random incidence, polar angle).
#include "device_util.h"

namespace rtmc {
namespace {

// Absolute margin of the node slab distances, per unit of coordinate
// magnitude and of |1/d|: 1.05 * 2^-20 (see slab_margins).
constexpr float kSlack = 1.05f / 1048576.0f;

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
// estimated remaining work, at least the idle lanes, at most claim_max): one
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
  // a small generation needs only its first ceil(count / 64) waves: each of
  // them claims until the counter runs out, so the others leave at once
  // instead of each paying one contended claim on the counter
  if ((uint64_t)(blockIdx.x * (uint32_t)wpb + (uint32_t)w) * 64u >= (uint64_t)count) return;
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
          claim = claim > a.claim_max ? a.claim_max : claim;
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

}  // namespace

// per wave: the stacks' LDS part, then the lanes' ray directions
size_t traverse_lds_bytes(int lds_stack, int block) { return (size_t)(block / 64) * (lds_stack + 3) * 64 * 4; }

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

}  // namespace rtmc
