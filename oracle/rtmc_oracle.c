/*
 * FP64 brute-force oracle for the ray-tracing Monte Carlo (RTMC) method of
 * Alvarado, Chang, Nadvornick, Ghoniem and Marian, "Monte Carlo raytracing
 * method for calculating secondary electron emission from micro-architected
 * surfaces" (arXiv 1806.00205).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code with the GPU library.
 *
 * What it computes, and where the paper defines it:
 *   - ray / triangle intersection by the Moller-Trumbore Cramer's-rule solve
 *     (section 2.1, Eqs. MT1-MT2 and the Cramer solution), scanning every
 *     triangle (the brute-force scan of section 2.1), with back-face culling,
 *     the parallel-ray check, the barycentric test and closest-hit selection
 *     (the four checks listed in section 2.1);
 *   - the local incidence angle and the sampling of the number, energy and
 *     direction of secondary rays from flat-surface tables (section 2.2);
 *   - the per-primary tree of branches, periodic x/y boundaries, the flat
 *     substrate and the escape test at z_max (section 2.2, Fig. flow);
 *   - the yield as escaped tracks per primary track (section 1, Fig. flow).
 *
 * Readings taken where the paper is silent or garbled (all in FP64 here):
 *   - Cramer denominator: det = (D x L2) . L1, the determinant of
 *     [-D, L1, L2]; the printed (D x L2) . L2 is identically zero.
 *   - barycentric limits: u >= 0, v >= 0, u + v <= 1 (the printed
 *     u^2 + v^2 <= 1 does not bound the triangle of Eq. MT2).
 *   - culling and the parallel check are one test: det > 1e-12 |L1||L2||D|;
 *     for counter-clockwise (outward) triangles det = -(D . s) so a positive
 *     det is a front-facing ray.
 *   - closest hit: lexicographic minimum of (t, triangle id), accepting
 *     0 < t <= distance to the cell boundary.
 *   - incidence angle: alpha = acos(|D . n|) in degrees, in [0, 90].
 *   - yield rounding: floor(delta) plus one with probability frac(delta)
 *     (the footnote of section 2.2).
 *   - secondary energies: inverse of the tabulated piecewise-linear CDF,
 *     truncated to the energy still available from the parent, so the
 *     daughters never carry more than the parent.
 *   - directions: cosine law about the element normal (sin^2 beta uniform),
 *     azimuth uniform; frame by the branchless construction of Duff et al.
 *     (JCGT 2017).
 *   - the paper's own emission rule (section 2.2, emission mode 1): a lone
 *     daughter gets E_SEE(E, alpha) and a cosine-law direction; a pair
 *     shares one xi: E1 = E_SEE sqrt(xi) at sin^2 beta1 = xi, E2 = cos^2
 *     beta1 E_SEE at beta2 = pi/2 - beta1; azimuths uniform and independent.
 *     More than two daughters (the fit exceeds 2 only outside 50-1000 eV)
 *     come in further pairs, an odd one last by the lone rule.  Each
 *     energy is clamped to [0, energy still available] (the fits go
 *     negative at low E and above the parent at high E).  Draw 2 + d serves
 *     daughter d (xi of a pair from its first daughter's draw, word 1).
 *   - E_c only stops re-emission at a hit; every daughter is traced.
 *   - a ray of generation max_gen that hits is absorbed without emission.
 *   - primaries start at a uniform point of the top face z_max; azimuth
 *     uniform; theta fixed, or uniform in [0, |theta|] when theta < 0.
 *   - absorption depth (section 3.2, Fig. pen, penetration profile): every ray of
 *     any generation that ends on a surface (triangle or substrate) is one
 *     absorption event at depth (z_max - z) / (z_max - z_min) in [0, 1].
 *   - random numbers: Philox4x32-10 (Salmon et al., SC'11), key = seed,
 *     counter = (primary id low, primary id high, path code, draw), mapped
 *     to (0, 1] by ((u >> 8) + 1) * 2^-24.  Draw 0 is a primary's birth,
 *     draw 1 the daughter count at a hit, draw 2 + d daughter d.  A
 *     daughter's path code is parent * 8 + d + 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

#define ORC_PERIODIC_XY 1u
#define ORC_SUBSTRATE 2u

/* path outcomes */
#define OUT_HIT 0
#define OUT_ESCAPE 1
#define OUT_SUBSTRATE 2
#define OUT_BOTTOM 3
#define OUT_SIDE 4
#define OUT_WRAPCAP 5

#define ID_SUBSTRATE (-2)
#define ID_ESCAPE (-1)
#define ID_LOST (-3)

static const double DET_EPS = 1e-12;
static const double SPAWN_EPS = 1e-4;
static const int WRAP_MAX = 10000;
static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------ Philox */

static void philox_round(uint32_t c[4], const uint32_t k[2]) {
  uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  uint32_t n0 = hi1 ^ c[1] ^ k[0];
  uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
    philox_round(c, k);
  }
  memcpy(out, c, sizeof(c));
}

static void draw4(uint64_t seed, uint64_t pid, uint32_t path, uint32_t draw, double xi[4]) {
  uint32_t ctr[4] = {(uint32_t)pid, (uint32_t)(pid >> 32), path, draw};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t u[4];
  orc_philox4x32_10(ctr, key, u);
  for (int i = 0; i < 4; ++i) xi[i] = (double)((u[i] >> 8) + 1u) * (1.0 / 16777216.0);
}

/* ------------------------------------------------------------------ mesh */

typedef struct {
  double v0[3], v1[3], v2[3];
  int32_t id; /* index into the caller's triangle array */
} otri;

typedef struct {
  otri* t;
  int64_t n;
  int64_t dropped;
  double lo[3], hi[3];
  uint32_t flags;
} omesh;

static void sub3(const double a[3], const double b[3], double r[3]) {
  r[0] = a[0] - b[0];
  r[1] = a[1] - b[1];
  r[2] = a[2] - b[2];
}
static void cross3(const double a[3], const double b[3], double r[3]) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

/* Promote the float mesh to FP64 and drop triangles whose normal s is exactly
 * zero (no intersection test can accept them).  Returns ORC_EINVAL on bad
 * indices, non-finite coordinates, vertices outside the box or a triangle
 * lying in a face of the cell. */
static int mesh_build(omesh* m, const float* verts, int64_t nv, const int32_t* tris, int64_t nt,
                      const double lo[3], const double hi[3], uint32_t flags) {
  memset(m, 0, sizeof(*m));
  for (int a = 0; a < 3; ++a) {
    m->lo[a] = lo[a];
    m->hi[a] = hi[a];
    if (!(hi[a] > lo[a])) return ORC_EINVAL;
  }
  m->flags = flags;
  if (nt < 0 || nv < 0) return ORC_EINVAL;
  for (int64_t i = 0; i < nv * 3; ++i) {
    if (!isfinite(verts[i])) return ORC_EINVAL;
    double x = verts[i];
    int a = (int)(i % 3);
    if (x < lo[a] || x > hi[a]) return ORC_EINVAL;
  }
  m->t = (otri*)malloc(sizeof(otri) * (size_t)(nt > 0 ? nt : 1));
  if (!m->t) return ORC_ENOMEM;
  for (int64_t j = 0; j < nt; ++j) {
    for (int k = 0; k < 3; ++k)
      if (tris[3 * j + k] < 0 || tris[3 * j + k] >= nv) {
        free(m->t);
        m->t = NULL;
        return ORC_EINVAL;
      }
    otri T;
    for (int a = 0; a < 3; ++a) {
      T.v0[a] = verts[3 * (int64_t)tris[3 * j + 0] + a];
      T.v1[a] = verts[3 * (int64_t)tris[3 * j + 1] + a];
      T.v2[a] = verts[3 * (int64_t)tris[3 * j + 2] + a];
    }
    double l1[3], l2[3], s[3];
    sub3(T.v1, T.v0, l1);
    sub3(T.v2, T.v0, l2);
    cross3(l1, l2, s);
    if (s[0] == 0.0 && s[1] == 0.0 && s[2] == 0.0) {
      m->dropped++;
      continue;
    }
    /* a surface lying in a face of the cell would be met exactly where the
       ray leaves the cell (periodic re-entry, the substrate plane, escape),
       and which of the two comes first is a matter of rounding: rejected */
    for (int a = 0; a < 3; ++a) {
      const int on_lo = T.v0[a] == lo[a] && T.v1[a] == lo[a] && T.v2[a] == lo[a];
      const int on_hi = T.v0[a] == hi[a] && T.v1[a] == hi[a] && T.v2[a] == hi[a];
      if (on_lo || on_hi) {
        free(m->t);
        m->t = NULL;
        return ORC_EINVAL;
      }
    }
    T.id = (int32_t)j;
    m->t[m->n++] = T;
  }
  return ORC_OK;
}

/* Closest front-facing triangle with 0 < t <= tmax: the brute-force scan of
 * section 2.1 solved by Cramer's rule. */
static int64_t seg_hit(const omesh* m, const double O[3], const double D[3], double tmax, double* t_out,
                       double* u_out, double* v_out, uint64_t* ntests) {
  int64_t best = -1;
  double bt = tmax, bu = 0, bv = 0;
  double dn = norm3(D);
  for (int64_t j = 0; j < m->n; ++j) {
    const otri* T = &m->t[j];
    double L1[3], L2[3], P[3], Tv[3], Q[3];
    sub3(T->v1, T->v0, L1);
    sub3(T->v2, T->v0, L2);
    cross3(D, L2, P);
    double det = dot3(P, L1);
    /* back-face culling and the parallel check */
    if (det <= DET_EPS * norm3(L1) * norm3(L2) * dn) continue;
    sub3(O, T->v0, Tv);
    double u = dot3(P, Tv) / det;
    if (u < 0.0 || u > 1.0) continue;
    cross3(Tv, L1, Q);
    double v = dot3(Q, D) / det;
    if (v < 0.0 || u + v > 1.0) continue;
    double t = dot3(Q, L2) / det;
    if (!(t > 0.0) || t > tmax) continue;
    if (best < 0 || t < bt || (t == bt && T->id < m->t[best].id)) {
      best = j;
      bt = t;
      bu = u;
      bv = v;
    }
  }
  *ntests += (uint64_t)m->n;
  *t_out = bt;
  *u_out = bu;
  *v_out = bv;
  return best;
}

typedef struct {
  int kind;
  int64_t tri; /* index into m->t when kind == OUT_HIT */
  double t_total;
  double P[3]; /* hit point (OUT_HIT / OUT_SUBSTRATE) */
  double n[3]; /* unit normal at the hit */
  double D[3];
  int wraps;
} opath;

/* Follow a ray through the periodic cell until it hits a surface, escapes
 * through z_max or is lost. */
static void trace_path(const omesh* m, const double O[3], const double D[3], opath* r, uint64_t* ntests) {
  double o[3] = {O[0], O[1], O[2]};
  double total = 0.0;
  int wraps = 0;
  const int periodic = (m->flags & ORC_PERIODIC_XY) != 0;
  memcpy(r->D, D, sizeof(double) * 3);
  for (;;) {
    double te[3];
    for (int a = 0; a < 3; ++a) {
      if (D[a] > 0.0)
        te[a] = (m->hi[a] - o[a]) / D[a];
      else if (D[a] < 0.0)
        te[a] = (m->lo[a] - o[a]) / D[a];
      else
        te[a] = INFINITY;
      if (te[a] < 0.0) te[a] = 0.0;
    }
    double texit = te[0];
    if (te[1] < texit) texit = te[1];
    if (te[2] < texit) texit = te[2];
    double t, u, v;
    int64_t j = seg_hit(m, o, D, texit, &t, &u, &v, ntests);
    if (j >= 0) {
      const otri* T = &m->t[j];
      for (int a = 0; a < 3; ++a) r->P[a] = (1.0 - u - v) * T->v0[a] + u * T->v1[a] + v * T->v2[a];
      double l1[3], l2[3], s[3];
      sub3(T->v1, T->v0, l1);
      sub3(T->v2, T->v0, l2);
      cross3(l1, l2, s);
      double sn = norm3(s);
      for (int a = 0; a < 3; ++a) r->n[a] = s[a] / sn;
      r->kind = OUT_HIT;
      r->tri = j;
      r->t_total = total + t;
      r->wraps = wraps;
      return;
    }
    if (te[2] <= te[0] && te[2] <= te[1]) {
      r->t_total = total + te[2];
      r->wraps = wraps;
      r->tri = -1;
      if (D[2] > 0.0) {
        r->kind = OUT_ESCAPE;
      } else if (m->flags & ORC_SUBSTRATE) {
        r->kind = OUT_SUBSTRATE;
        r->P[0] = o[0] + te[2] * D[0];
        r->P[1] = o[1] + te[2] * D[1];
        r->P[2] = m->lo[2];
        r->n[0] = 0.0;
        r->n[1] = 0.0;
        r->n[2] = 1.0;
      } else {
        r->kind = OUT_BOTTOM;
      }
      return;
    }
    if (!periodic) {
      r->kind = OUT_SIDE;
      r->tri = -1;
      r->t_total = total + texit;
      r->wraps = wraps;
      return;
    }
    /* periodic re-entry through the opposite x / y face */
    total += texit;
    double p[3];
    for (int a = 0; a < 3; ++a) p[a] = o[a] + texit * D[a];
    for (int a = 0; a < 2; ++a) {
      if (te[a] == texit)
        p[a] = D[a] > 0.0 ? m->lo[a] : m->hi[a];
      else if (p[a] < m->lo[a])
        p[a] = m->lo[a];
      else if (p[a] > m->hi[a])
        p[a] = m->hi[a];
    }
    if (p[2] < m->lo[2]) p[2] = m->lo[2];
    if (p[2] > m->hi[2]) p[2] = m->hi[2];
    memcpy(o, p, sizeof(p));
    if (++wraps > WRAP_MAX) {
      r->kind = OUT_WRAPCAP;
      r->tri = -1;
      r->t_total = total;
      r->wraps = wraps;
      return;
    }
  }
}

/* ------------------------------------------------------------------ tables */

typedef struct {
  const float* yld; /* [nE][nth] */
  int32_t nE, nth;
  double Emin, Emax;
  const float* cdfE;
  const float* cdfF;
  int32_t ncdf;
  double Ec;
  const float* esee;
  int32_t emission;
} otab;

/* Table value at (E, alpha): bilinear in (ln E, alpha) on the grid, clamped. */
static double tab_grid(const otab* T, const float* tbl, double E, double alpha) {
  double x = (log(E) - log(T->Emin)) / (log(T->Emax) - log(T->Emin)) * (T->nE - 1);
  if (x < 0.0) x = 0.0;
  if (x > T->nE - 1) x = T->nE - 1;
  int i = (int)floor(x);
  if (i > T->nE - 2) i = T->nE - 2;
  double fx = x - i;
  double y = alpha / 90.0 * (T->nth - 1);
  if (y < 0.0) y = 0.0;
  if (y > T->nth - 1) y = T->nth - 1;
  int j = (int)floor(y);
  if (j > T->nth - 2) j = T->nth - 2;
  double fy = y - j;
  double y00 = tbl[(int64_t)i * T->nth + j], y10 = tbl[(int64_t)(i + 1) * T->nth + j];
  double y01 = tbl[(int64_t)i * T->nth + j + 1], y11 = tbl[(int64_t)(i + 1) * T->nth + j + 1];
  return (1 - fx) * (1 - fy) * y00 + fx * (1 - fy) * y10 + (1 - fx) * fy * y01 + fx * fy * y11;
}

static double tab_yield(const otab* T, double E, double alpha) { return tab_grid(T, T->yld, E, alpha); }

/* Piecewise-linear CDF through the tabulated points. */
static double tab_cdf(const otab* T, double E) {
  if (E <= T->cdfE[0]) return T->cdfF[0];
  for (int k = 0; k + 1 < T->ncdf; ++k) {
    double e0 = T->cdfE[k], e1 = T->cdfE[k + 1];
    if (E < e1) return T->cdfF[k] + (E - e0) / (e1 - e0) * ((double)T->cdfF[k + 1] - T->cdfF[k]);
  }
  return T->cdfF[T->ncdf - 1];
}

/* Inverse of the piecewise-linear CDF: the energy where it reaches c. */
static double tab_cdf_inv(const otab* T, double c) {
  for (int k = 0; k + 1 < T->ncdf; ++k) {
    double f0 = T->cdfF[k], f1 = T->cdfF[k + 1];
    if (f1 >= c) {
      if (f1 <= f0) return T->cdfE[k];
      return T->cdfE[k] + (c - f0) / (f1 - f0) * ((double)T->cdfE[k + 1] - T->cdfE[k]);
    }
  }
  return T->cdfE[T->ncdf - 1];
}

/* Orthonormal frame (t1, t2) completing unit n (Duff et al., JCGT 2017). */
static void onb(const double n[3], double t1[3], double t2[3]) {
  double sign = copysign(1.0, n[2]);
  double a = -1.0 / (sign + n[2]);
  double b = n[0] * n[1] * a;
  t1[0] = 1.0 + sign * n[0] * n[0] * a;
  t1[1] = sign * b;
  t1[2] = -sign * n[0];
  t2[0] = b;
  t2[1] = sign + n[1] * n[1] * a;
  t2[2] = -n[1];
}

/* ------------------------------------------------------------------ public */

typedef struct {
  const float* verts;
  int64_t n_verts;
  const int32_t* tris;
  int64_t n_tris;
  double lo[3], hi[3];
  uint32_t flags;
} orc_mesh_in;

typedef struct {
  const float* yld;
  int32_t n_E, n_theta;
  double E_min, E_max;
  const float* cdf_E;
  const float* cdf_F;
  int32_t n_cdf;
  double Ec;
  const float* esee; /* E_SEE on the yield grid (emission 1), else unused */
  int32_t emission;  /* 0: spectrum (CDF) + cosine law; 1: the paper's one/two-daughter rule */
} orc_tables_in;

typedef struct {
  double E0;
  double theta_deg; /* < 0: uniform in [0, -theta_deg] */
  uint64_t pid0;    /* first primary id */
  uint64_t n_primaries;
  uint64_t seed;
  int32_t max_gen;
  int32_t n_ebins; /* escaped-energy histogram over [0, E0] */
  int32_t n_abins; /* escape polar-angle histogram over [0, 90) deg */
  int32_t n_threads;
  int32_t n_zbins; /* absorption-depth histogram over [0, 1] (0: none) */
} orc_job;

typedef struct {
  uint64_t n_primaries, n_rays, n_escaped, n_absorbed, n_truncated, n_lost;
  uint64_t n_substrate, n_wraps, n_tri_tests, n_dropped_tris;
  double e_escaped, e_deposited, yield, yield_sigma;
} orc_result;

int orc_mesh_dropped(const orc_mesh_in* mi, int64_t* dropped) {
  omesh m;
  int st = mesh_build(&m, mi->verts, mi->n_verts, mi->tris, mi->n_tris, mi->lo, mi->hi, mi->flags);
  if (st) return st;
  *dropped = m.dropped;
  free(m.t);
  return ORC_OK;
}

/* First surface reached by each ray, following periodic re-entry.  rays is
 * [n][6] (origin, direction).  tri_out receives the caller's triangle index,
 * or -1 (escape through z_max), -2 (substrate), -3 (lost).  t_out receives
 * the path length along the ray over all periodic segments. */
int orc_first_hit(const orc_mesh_in* mi, const double* rays, int64_t n, int32_t* tri_out, double* t_out,
                  int32_t* wraps_out, int32_t n_threads) {
  omesh m;
  int st = mesh_build(&m, mi->verts, mi->n_verts, mi->tris, mi->n_tris, mi->lo, mi->hi, mi->flags);
  if (st) return st;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    uint64_t tests = 0;
    opath r;
    trace_path(&m, rays + 6 * i, rays + 6 * i + 3, &r, &tests);
    int32_t id;
    if (r.kind == OUT_HIT)
      id = m.t[r.tri].id;
    else if (r.kind == OUT_ESCAPE)
      id = ID_ESCAPE;
    else if (r.kind == OUT_SUBSTRATE)
      id = ID_SUBSTRATE;
    else
      id = ID_LOST;
    tri_out[i] = id;
    t_out[i] = r.t_total;
    if (wraps_out) wraps_out[i] = r.wraps;
  }
  free(m.t);
  return ORC_OK;
}

typedef struct {
  double o[3], d[3], E;
  uint32_t path;
  int32_t gen;
} oray;

/* Full RTMC over primaries pid0 .. pid0 + n - 1.  Per-primary arrays
 * (escape count, escaped energy, deposited energy, rays) are optional. */
int orc_trace(const orc_mesh_in* mi, const orc_tables_in* ti, const orc_job* job, orc_result* res,
              uint64_t* e_hist, uint64_t* a_hist, uint64_t* z_hist, uint32_t* pp_escaped, double* pp_e_esc,
              double* pp_e_dep, uint32_t* pp_rays) {
  if (job->max_gen < 0 || job->max_gen > 10 || !(job->E0 > 0.0) || job->n_ebins < 1 || job->n_abins < 1 ||
      job->n_zbins < 0 || (job->n_zbins > 0 && !z_hist))
    return ORC_EINVAL;
  if (ti->n_E < 2 || ti->n_theta < 2 || ti->n_cdf < 2) return ORC_EINVAL;
  omesh m;
  int st = mesh_build(&m, mi->verts, mi->n_verts, mi->tris, mi->n_tris, mi->lo, mi->hi, mi->flags);
  if (st) return st;
  if (ti->emission < 0 || ti->emission > 1 || (ti->emission == 1 && !ti->esee)) return ORC_EINVAL;
  otab T = {ti->yld, ti->n_E, ti->n_theta, ti->E_min, ti->E_max, ti->cdf_E, ti->cdf_F, ti->n_cdf, ti->Ec,
            ti->esee, ti->emission};
  const int nthreads_req = job->n_threads;
#ifdef _OPENMP
  if (nthreads_req > 0) omp_set_num_threads(nthreads_req);
#endif
  const int NE = job->n_ebins, NA = job->n_abins, NZ = job->n_zbins;
  uint64_t g_rays = 0, g_esc = 0, g_abs = 0, g_trunc = 0, g_lost = 0, g_sub = 0, g_wraps = 0, g_tests = 0;
  double g_eesc = 0.0, g_edep = 0.0, g_c2 = 0.0;
  memset(e_hist, 0, sizeof(uint64_t) * NE);
  memset(a_hist, 0, sizeof(uint64_t) * NA);
  if (NZ) memset(z_hist, 0, sizeof(uint64_t) * NZ);
  int failed = 0;
#pragma omp parallel
  {
    uint64_t l_rays = 0, l_esc = 0, l_abs = 0, l_trunc = 0, l_lost = 0, l_sub = 0, l_wraps = 0, l_tests = 0;
    double l_eesc = 0.0, l_edep = 0.0, l_c2 = 0.0;
    uint64_t* lh_e = (uint64_t*)calloc((size_t)NE, sizeof(uint64_t));
    uint64_t* lh_a = (uint64_t*)calloc((size_t)NA, sizeof(uint64_t));
    uint64_t* lh_z = (uint64_t*)calloc((size_t)(NZ > 0 ? NZ : 1), sizeof(uint64_t));
    size_t cap = 64;
    oray* q = (oray*)malloc(sizeof(oray) * cap);
    if (!lh_e || !lh_a || !lh_z || !q) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp for schedule(dynamic, 4)
    for (uint64_t k = 0; k < job->n_primaries; ++k) {
      if (failed) continue;
      const uint64_t pid = job->pid0 + k;
      double xi[4];
      draw4(job->seed, pid, 0u, 0u, xi);
      double th = job->theta_deg >= 0.0 ? job->theta_deg : -job->theta_deg * xi[3];
      double thr = th * PI / 180.0, psi = 2.0 * PI * xi[2];
      oray r0;
      r0.o[0] = m.lo[0] + (m.hi[0] - m.lo[0]) * xi[0];
      r0.o[1] = m.lo[1] + (m.hi[1] - m.lo[1]) * xi[1];
      r0.o[2] = m.hi[2];
      r0.d[0] = sin(thr) * cos(psi);
      r0.d[1] = sin(thr) * sin(psi);
      r0.d[2] = -cos(thr);
      r0.E = job->E0;
      r0.path = 0;
      r0.gen = 0;
      /* the tree of branches, processed first in, first out */
      size_t head = 0, tail = 0;
      q[tail++] = r0;
      uint32_t c_esc = 0, c_rays = 0;
      double e_esc = 0.0, e_dep = 0.0;
      while (head < tail) {
        oray ray = q[head++];
        c_rays++;
        opath p;
        trace_path(&m, ray.o, ray.d, &p, &l_tests);
        l_wraps += (uint64_t)p.wraps;
        if (p.kind == OUT_ESCAPE) {
          c_esc++;
          e_esc += ray.E;
          int eb = (int)floor(ray.E / job->E0 * NE);
          if (eb < 0) eb = 0;
          if (eb > NE - 1) eb = NE - 1;
          lh_e[eb]++;
          double dz = ray.d[2] > 1.0 ? 1.0 : ray.d[2];
          double pol = acos(dz) * 180.0 / PI;
          int ab = (int)floor(pol / 90.0 * NA);
          if (ab < 0) ab = 0;
          if (ab > NA - 1) ab = NA - 1;
          lh_a[ab]++;
          continue;
        }
        if (p.kind != OUT_HIT && p.kind != OUT_SUBSTRATE) {
          l_lost++;
          e_dep += ray.E;
          continue;
        }
        if (p.kind == OUT_SUBSTRATE) l_sub++;
        if (NZ) {
          /* the ray ends on a surface: its depth below the top of the cell,
             as a fraction of the cell height (section 3.2, Fig. pen, penetration) */
          int zb = (int)floor((m.hi[2] - p.P[2]) / (m.hi[2] - m.lo[2]) * NZ);
          if (zb < 0) zb = 0;
          if (zb > NZ - 1) zb = NZ - 1;
          lh_z[zb]++;
        }
        if (ray.gen >= job->max_gen) {
          l_trunc++;
          e_dep += ray.E;
          continue;
        }
        l_abs++;
        if (ray.E <= T.Ec) {
          e_dep += ray.E;
          continue;
        }
        double cosa = -dot3(ray.d, p.n);
        if (cosa > 1.0) cosa = 1.0;
        if (cosa < 0.0) cosa = 0.0;
        double alpha = acos(cosa) * 180.0 / PI;
        double delta = tab_yield(&T, ray.E, alpha);
        double u1[4];
        draw4(job->seed, pid, ray.path, 1u, u1);
        double fl = floor(delta);
        int nd = (int)fl + (u1[0] < delta - fl ? 1 : 0);
        double Eav = ray.E;
        /* the paper's rule (section 2.2): E_SEE at (E, alpha) from its table */
        const double es = T.emission == 1 ? tab_grid(&T, T.esee, ray.E, alpha) : 0.0;
        double xi_pair = 0.0;
        for (int d = 0; d < nd; ++d) {
          double u[4];
          draw4(job->seed, pid, ray.path, 2u + (uint32_t)d, u);
          double Ed, s2; /* energy and sin^2 of the polar angle about the normal */
          if (T.emission == 0) {
            Ed = tab_cdf_inv(&T, u[0] * tab_cdf(&T, Eav));
            s2 = u[1];
          } else if (d % 2 == 1) {
            /* second of a pair: beta2 = pi/2 - beta1, E2 = cos^2(beta1) E_SEE */
            Ed = (1.0 - xi_pair) * es;
            s2 = 1.0 - xi_pair;
          } else if (d + 1 < nd) {
            /* first of a pair: E1 = E_SEE sqrt(xi), beta1 = asin(sqrt(xi)) */
            xi_pair = u[1];
            Ed = es * sqrt(xi_pair);
            s2 = xi_pair;
          } else {
            /* a lone daughter: energy E_SEE, cosine-law direction */
            Ed = es;
            s2 = u[1];
          }
          if (Ed < 0.0) Ed = 0.0;
          if (Ed > Eav) Ed = Eav;
          Eav -= Ed;
          double sb = sqrt(s2), cb = sqrt(1.0 - s2), ph = 2.0 * PI * u[2];
          double t1[3], t2[3];
          onb(p.n, t1, t2);
          oray dr;
          for (int a = 0; a < 3; ++a) {
            dr.d[a] = cb * p.n[a] + sb * (cos(ph) * t1[a] + sin(ph) * t2[a]);
            dr.o[a] = p.P[a] + SPAWN_EPS * p.n[a];
          }
          if (m.flags & ORC_PERIODIC_XY) {
            for (int a = 0; a < 2; ++a) {
              double L = m.hi[a] - m.lo[a];
              if (dr.o[a] > m.hi[a]) dr.o[a] -= L;
              if (dr.o[a] < m.lo[a]) dr.o[a] += L;
            }
          }
          if (dr.o[2] > m.hi[2]) dr.o[2] = m.hi[2];
          if (dr.o[2] < m.lo[2]) dr.o[2] = m.lo[2];
          dr.E = Ed;
          dr.path = ray.path * 8u + (uint32_t)d + 1u;
          dr.gen = ray.gen + 1;
          if (tail == cap) {
            /* compact the consumed prefix, then grow */
            memmove(q, q + head, sizeof(oray) * (tail - head));
            tail -= head;
            head = 0;
            if (tail == cap) {
              cap *= 2;
              oray* nq = (oray*)realloc(q, sizeof(oray) * cap);
              if (!nq) {
                failed = 1;
                break;
              }
              q = nq;
            }
          }
          q[tail++] = dr;
        }
        e_dep += Eav;
      }
      l_rays += c_rays;
      l_esc += c_esc;
      l_eesc += e_esc;
      l_edep += e_dep;
      l_c2 += (double)c_esc * (double)c_esc;
      if (pp_escaped) pp_escaped[k] = c_esc;
      if (pp_e_esc) pp_e_esc[k] = e_esc;
      if (pp_e_dep) pp_e_dep[k] = e_dep;
      if (pp_rays) pp_rays[k] = c_rays;
    }
#pragma omp critical
    {
      g_rays += l_rays;
      g_esc += l_esc;
      g_abs += l_abs;
      g_trunc += l_trunc;
      g_lost += l_lost;
      g_sub += l_sub;
      g_wraps += l_wraps;
      g_tests += l_tests;
      g_eesc += l_eesc;
      g_edep += l_edep;
      g_c2 += l_c2;
      if (lh_e)
        for (int b = 0; b < NE; ++b) e_hist[b] += lh_e[b];
      if (lh_a)
        for (int b = 0; b < NA; ++b) a_hist[b] += lh_a[b];
      if (lh_z)
        for (int b = 0; b < NZ; ++b) z_hist[b] += lh_z[b];
    }
    free(lh_e);
    free(lh_a);
    free(lh_z);
    free(q);
  }
  free(m.t);
  if (failed) return ORC_ENOMEM;
  memset(res, 0, sizeof(*res));
  res->n_primaries = job->n_primaries;
  res->n_rays = g_rays;
  res->n_escaped = g_esc;
  res->n_absorbed = g_abs;
  res->n_truncated = g_trunc;
  res->n_lost = g_lost;
  res->n_substrate = g_sub;
  res->n_wraps = g_wraps;
  res->n_tri_tests = g_tests;
  res->n_dropped_tris = (uint64_t)m.dropped;
  res->e_escaped = g_eesc;
  res->e_deposited = g_edep;
  double N = (double)job->n_primaries;
  if (N > 0) {
    double mean = (double)g_esc / N;
    res->yield = mean;
    double var = N > 1 ? (g_c2 - N * mean * mean) / (N - 1.0) : 0.0;
    if (var < 0) var = 0;
    res->yield_sigma = sqrt(var / N);
  }
  return ORC_OK;
}

/* Table look-ups exposed for the tests. */
double orc_table_yield(const orc_tables_in* ti, double E, double alpha) {
  otab T = {ti->yld, ti->n_E, ti->n_theta, ti->E_min, ti->E_max, ti->cdf_E, ti->cdf_F, ti->n_cdf, ti->Ec};
  return tab_yield(&T, E, alpha);
}

double orc_sample_energy(const orc_tables_in* ti, double xi, double E_avail) {
  otab T = {ti->yld, ti->n_E, ti->n_theta, ti->E_min, ti->E_max, ti->cdf_E, ti->cdf_F, ti->n_cdf, ti->Ec};
  double e = tab_cdf_inv(&T, xi * tab_cdf(&T, E_avail));
  return e > E_avail ? E_avail : e;
}

void orc_onb(const double n[3], double t1[3], double t2[3]) { onb(n, t1, t2); }
