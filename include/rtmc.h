/*
 * rtmc.h -- C interface of the MI355X (gfx950) ray-tracing Monte Carlo
 * library for secondary electron emission from triangulated porous surfaces.
 *
 * Method: Alvarado, Chang, Nadvornick, Ghoniem and Marian, "Monte Carlo
 * raytracing method for calculating secondary electron emission from
 * micro-architected surfaces" (arXiv 1806.00205).  Primary electron rays
 * enter a periodic surface mesh from above (section 2, Fig. flow); each hit
 * on a surface element (section 2.1) samples the number, energy and
 * direction of secondary rays from flat-surface tables (section 2.2); every
 * ray is followed until it is reabsorbed or escapes through z_max, and the
 * yield is escaped rays per primary (section 1, Fig. flow).
 *
 * Conventions shared by every call:
 *   - Every call returns rtmc_status.  On failure the context keeps a
 *     message, read with rtmc_last_error(); nothing is thrown across the
 *     interface.  Calls made in the wrong order return RTMC_ESTATE.
 *   - Host arrays passed in are copied before the call returns; the caller
 *     keeps ownership.  Pointers documented as "device" must point to GPU
 *     memory on the context's device, and are only read or written by work
 *     enqueued on the context's stream.
 *   - Device memory owned by the library is obtained from the allocator
 *     given to rtmc_create (hipMalloc when none) and released by
 *     rtmc_destroy.
 *   - All work is enqueued on the context's stream.  rtmc_trace,
 *     rtmc_trace_batch and rtmc_build_bvh synchronise that stream before
 *     returning; rtmc_first_hit and rtmc_sort_pairs_u64 do not.
 *   - Units: energies in eV, angles in degrees, lengths in mesh units.
 *   - A context is not thread-safe: use one per host thread.
 */
#ifndef RTMC_H
#define RTMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rtmc_ctx rtmc_ctx;

typedef enum {
  RTMC_OK = 0,
  RTMC_EINVAL = -1,    /* bad argument: sizes, ids, non-finite values */
  RTMC_ENOMEM = -2,    /* device allocation failed */
  RTMC_EDEVICE = -3,   /* a HIP call failed */
  RTMC_ESTATE = -4,    /* call out of order (e.g. trace before the BVH) */
  RTMC_EOVERFLOW = -5, /* a single primary's ray tree exceeded the queue */
  RTMC_ENOTIMPL = -6
} rtmc_status;

/* scene flags */
#define RTMC_PERIODIC_XY 1u /* x and y wrap around (section 2.2) */
#define RTMC_SUBSTRATE 2u   /* emitting flat plane at z_min, normal +z (section 2.2) */

/* first-hit codes besides triangle indices */
#define RTMC_HIT_ESCAPE (-1)    /* left through z_max moving up */
#define RTMC_HIT_SUBSTRATE (-2) /* reached the substrate plane */
#define RTMC_HIT_LOST (-3)      /* left through a non-periodic side or the open bottom, or wrapped too often */

typedef struct {
  void* (*alloc)(size_t bytes, void* user); /* returns device memory or NULL */
  void (*free)(void* ptr, void* user);
  void* user;
} rtmc_allocator;

/* Flat-surface tables (section 2.2): the yield and the secondary-energy
 * spectrum of an ideally flat surface, computed beforehand.
 *   yield[i * n_theta + j]: yield at E_i = E_min * (E_max / E_min)^(i / (n_E - 1))
 *       and local incidence angle alpha_j = 90 j / (n_theta - 1); looked up
 *       bilinearly in (ln E, alpha) and clamped at the grid edges.  Values in
 *       [0, 7).  2 <= n_E, 2 <= n_theta, n_E * n_theta <= 8192.
 *   cdf_E[k], cdf_F[k]: the secondary-energy CDF as points; cdf_E strictly
 *       increasing from 0, cdf_F nondecreasing from 0 to 1.  The spectrum is
 *       the piecewise-linear CDF through them.  2 <= n_cdf <= 1024.
 *   Ec: emission cut-off (work function + Fermi energy, section 2.2): a ray
 *       with E <= Ec that hits a surface emits nothing.
 *   emission: how daughters get energies and directions.
 *     RTMC_EMIT_SPECTRUM: energies from the CDF above, each truncated to the
 *       energy the parent still has; directions by the cosine law.
 *     RTMC_EMIT_PAPER: the paper's rule (section 2.2) with E_SEE from esee:
 *       a lone daughter takes E_SEE and a cosine-law direction; a pair
 *       shares one xi, E1 = E_SEE sqrt(xi) at sin^2 beta1 = xi and E2 =
 *       cos^2 beta1 E_SEE at beta2 = pi/2 - beta1; further daughters come in
 *       pairs, an odd one last alone; every energy is clamped to [0, energy
 *       still available].  Azimuths are uniform.
 *   esee[i * n_theta + j]: E_SEE (eV) on the yield grid, finite, looked up
 *       like the yield; required for RTMC_EMIT_PAPER, else may be NULL.
 * All arrays are host memory, copied. */
#define RTMC_EMIT_SPECTRUM 0
#define RTMC_EMIT_PAPER 1
typedef struct {
  int32_t n_E, n_theta;
  double E_min, E_max;
  const float* yield;
  int32_t n_cdf;
  const float* cdf_E;
  const float* cdf_F;
  double Ec;
  const float* esee;
  int32_t emission;
} rtmc_tables;

/* Options of one trace.  NULL selects max_gen 6, 256 energy bins, 90 angle
 * bins, pid0 0 and no outputs beyond *out. */
typedef struct {
  int32_t max_gen;       /* deepest generation, 0..10 (primaries are generation 0); a ray of
                            this generation that hits is absorbed without emission */
  int32_t n_ebins;       /* escaped-energy histogram bins over [0, E0]; 0 means 256; <= 1024 */
  int32_t n_abins;       /* escape polar-angle histogram bins over [0, 90) deg; 0 means 90; <= 360 */
  uint64_t pid0;         /* first primary id (resume: [0,k) + [k,N) equals [0,N)); pid0 + n < 2^32 */
  uint64_t* e_hist;      /* host, n_ebins counts, may be NULL */
  uint64_t* a_hist;      /* host, n_abins counts, may be NULL */
  uint32_t* pp_escaped;  /* device, n_primaries escape counts indexed by primary id - pid0, may be NULL */
  int32_t n_zbins;       /* absorption-depth histogram (section 3.2, Fig. pen): every ray of any generation that
                            ends on a surface counts once at depth (z_max - z) / (z_max - z_min), in
                            n_zbins bins over [0, 1]; 0 means none; <= 256 */
  uint64_t* z_hist;      /* host, n_zbins counts, may be NULL */
  float* replay;         /* device float [n_replay * 6], may be NULL: the first n_replay rays of generation
                            replay_gen (daughters as spawned: origin, unit direction; first chunk only, in
                            queue order, which depends on scheduling) for re-tracing elsewhere */
  int64_t n_replay;      /* capacity of replay in rays, < 2^32 */
  int32_t replay_gen;    /* 1 .. max_gen when replay is set */
  int64_t* n_replay_out; /* host, may be NULL: how many rays were written to replay */
} rtmc_trace_opts;

typedef struct {
  double yield;        /* escaped rays / primaries */
  double yield_sigma;  /* standard error from the per-primary escape counts */
  uint64_t n_primaries, n_rays, n_escaped, n_absorbed, n_truncated, n_lost;
  uint64_t n_substrate, n_wraps, n_node_visits, n_tri_tests, n_spawned;
  double e_escaped;    /* summed energy of escaped rays (2^-20 eV fixed point, exact sums) */
  double e_deposited;  /* energy left in the surface (same fixed point); e_escaped + e_deposited = E0 n */
  double ms;           /* elapsed device time of the whole launch sequence */
  double kernel_ms;    /* summed duration of the traversal-kernel launches (HIP events around
                          each launch; 0 when rtmc_trace_batch replays a graph) */
  double shade_ms;     /* summed duration of the shading-kernel launches (same rules) */
  uint64_t n_kernel_launches;
  int32_t n_chunks;    /* primary chunks used (grows when a queue would overflow) */
} rtmc_result;

/* Launch shape of the traversal kernel (rtmc_autotune picks one). */
typedef struct {
  int32_t block;     /* threads per workgroup: 64..256, multiple of 64 */
  int32_t wg_per_cu; /* persistent workgroups per compute unit, >= 1 */
  int32_t lds_stack; /* traversal stack entries per lane held in LDS, 4..64 */
  int32_t chunk;     /* primaries per chunk; sizes the daughter queues */
  int32_t refill;    /* a wave fetches new rays once this many of its 64 lanes are idle, 1..64 */
  int32_t occupancy; /* traversal kernel build, waves per SIMD (registers capped to fit): 6 or 8;
                        any other value: 7 for one scene, 6 for a batch (the default) */
  int32_t claim;     /* rays per wave per claim: the largest block of a generation's rays one traversal
                        wave takes from the shared counter at once, 64..8192; 0 means 2048 */
} rtmc_launch_cfg;

typedef struct {
  int64_t n_tris_in, n_tris, n_dropped, n_nodes;
  int32_t bvh_built, bvh_depth;
  double lo[3], hi[3];
  uint32_t flags;
  double build_ms;
} rtmc_scene_info;

/* One (scene, energy, angle) point of a batched trace.  Its primaries have
 * ids 0 .. n_primaries - 1 and the random numbers of rtmc_trace with the same
 * seed, so a job reproduces the single trace of the same point. */
typedef struct {
  int32_t scene_id;
  double E_eV;
  double theta_deg;     /* >= 0 fixed incidence; < 0 uniform in [0, -theta_deg] */
  uint64_t n_primaries; /* < 2^32 */
  uint64_t seed;
  uint32_t* pp_escaped; /* device, n_primaries escape counts indexed by primary id, may be NULL */
} rtmc_job;

/* Create a context on HIP device `device`.  alloc may be NULL (hipMalloc);
 * hip_stream is a hipStream_t or NULL for the null stream. */
rtmc_status rtmc_create(rtmc_ctx** out, int device, const rtmc_allocator* alloc, void* hip_stream);

/* Free every device buffer of the context and the context itself. */
void rtmc_destroy(rtmc_ctx* ctx);

/* Message of the last failed call on ctx; valid until the next call. */
const char* rtmc_last_error(const rtmc_ctx* ctx);

/* Switch the stream later work is enqueued on. */
rtmc_status rtmc_set_stream(rtmc_ctx* ctx, void* hip_stream);

/* Surface mesh (section 2.1: triangles V0 V1 V2, normal (V1-V0) x (V2-V0)
 * pointing into the vacuum, i.e. counter-clockwise seen from the vacuum side).
 *   verts: host float [n_verts * 3]; tris: host int32 [n_tris * 3].
 *   box_lo/box_hi: the cell; x and y wrap around when RTMC_PERIODIC_XY is set;
 *   primaries start on z = box_hi[2]; box_lo[2] is the substrate plane.
 *   Every vertex must lie inside the box and be finite; every index in
 *   [0, n_verts).  Triangles whose normal is exactly zero are dropped and
 *   counted.  A triangle lying in a face of the box (all three vertices on
 *   box_lo[a], or all on box_hi[a], for some axis a) is refused with
 *   RTMC_EINVAL: a ray would meet it exactly where it leaves the cell, and
 *   which of the two comes first would be decided by rounding.  Returns the
 *   new scene id in *scene_id. */
rtmc_status rtmc_load_mesh(rtmc_ctx* ctx, const float* verts, int64_t n_verts, const int32_t* tris,
                           int64_t n_tris, const double box_lo[3], const double box_hi[3], uint32_t flags,
                           int32_t* scene_id);

/* Build the linear BVH of a scene on the device (Morton codes of triangle
 * centroids, radix sort, Karras hierarchy, bottom-up bounds).  The brute-force
 * scan of section 2.1 is what it replaces. */
rtmc_status rtmc_build_bvh(rtmc_ctx* ctx, int32_t scene_id);

rtmc_status rtmc_get_scene_info(rtmc_ctx* ctx, int32_t scene_id, rtmc_scene_info* out);

/* Copy a built BVH to host memory (structural checks).
 *   nodes: host float [n_nodes * 16]: per node the left child box (lo xyz,
 *          hi xyz), the right child box, then the two child links as int32
 *          bit patterns (bit 31 set: leaf, low bits: sorted triangle index).
 *   tris:  host float [n_tris * 12]: per sorted triangle V0, V1, V2 as
 *          (x, y, z, w) with w of V0 the caller's triangle index as int32 bits.
 *   Either may be NULL. */
rtmc_status rtmc_bvh_download(rtmc_ctx* ctx, int32_t scene_id, float* nodes, float* tris);

/* Copy the 4-wide nodes that traversal reads (for inspection and tests).
 * Each node holds the children of one binary node, the inner child of
 * largest surface area replaced by its two children until four slots are
 * filled.  Node 0 is the root (binary node 0); the nodes reached from it
 * follow level by level, the inner children of a node in consecutive nodes
 * (their order within a level may differ from build to build); the rest of
 * the n_nodes records are zero.  wide: host uint32 [n_nodes * 16]:
 *   words 0-2: float origin o (x, y, z); words 3, 14, 15: the per-axis
 *     scales s_x, s_y, s_z as floats, each a power of two;
 *   words 4-7: child links (bit 31 set: leaf, low bits: sorted triangle
 *     index; else a node index; 0xFFFFFFFF: unused slot);
 *   words 8-13: lo_x, lo_y, lo_z, hi_x, hi_y, hi_z, each four bytes q (byte j
 *     for child j); a bound decodes as fmaf(q, s, o) and contains the exact
 *     child box. */
rtmc_status rtmc_bvh_download_wide(rtmc_ctx* ctx, int32_t scene_id, uint32_t* wide);

/* Upload flat-surface tables; returns the table id in *table_id. */
rtmc_status rtmc_load_tables(rtmc_ctx* ctx, const rtmc_tables* t, int32_t* table_id);

/* Trace n_primaries primaries of energy E_eV at polar angle theta_deg (< 0:
 * uniform in [0, -theta_deg]) with random azimuth from uniform points of the
 * top face, following every secondary until it is absorbed or escapes
 * (Fig. flow).  Random numbers: Philox4x32-10 keyed by seed, counter
 * (primary id, 0, path code, draw).  Fills *out; histograms and per-primary
 * counts as requested in opts (may be NULL). */
rtmc_status rtmc_trace(rtmc_ctx* ctx, int32_t scene_id, int32_t table_id, double E_eV, double theta_deg,
                       uint64_t n_primaries, uint64_t seed, const rtmc_trace_opts* opts, rtmc_result* out);

/* Many (scene, E, theta) jobs through one launch sequence: chunks of the
 * concatenated primaries (at most the launch configuration's chunk; a chunk
 * holding a quarter of that is closed before it would span a 33rd job) go
 * through traversal and shading generation by generation; outs[i] receives job i's result.  One table set and max_gen
 * for all jobs.  A sequence of more than 128 traversal launches (chunks x
 * (max_gen + 1)) is replayed as a HIP graph, and kernel_ms / shade_ms are then
 * 0; a shorter one is launched directly and timed launch by launch.  Jobs
 * that share one scene run the single-scene traversal kernel.  Integer
 * tallies equal those of the same jobs traced one by one. */
rtmc_status rtmc_trace_batch(rtmc_ctx* ctx, int32_t table_id, const rtmc_job* jobs, int64_t n_jobs,
                             int32_t max_gen, rtmc_result* outs);

/* First surface reached by each ray, following periodic re-entry: the
 * closest front-facing element along the ray (the intersection checks of
 * section 2.1), or the substrate, or escape (section 2.2).
 *   rays: device float [n * 6] (origin xyz, unit direction xyz);
 *   tri_out: device int32 [n], the caller's triangle index or an RTMC_HIT_ code;
 *   t_out: device float [n], path length over all periodic segments.
 *   Asynchronous on the context stream. */
rtmc_status rtmc_first_hit(rtmc_ctx* ctx, int32_t scene_id, const float* rays, int64_t n, int32_t* tri_out,
                           float* t_out);

/* rtmc_first_hit for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, hosts that forbid allocation): the
 * same kernels and results as rtmc_first_hit, with every scratch buffer in a
 * fixed 32 MiB array that the library's code object holds on each GPU it
 * runs on, from the first rtmc_create on that GPU until the process ends.
 * The call allocates nothing and does not synchronise: it returns once its
 * kernels are enqueued on the context stream.
 *   rays, tri_out, t_out: as for rtmc_first_hit (device memory, caller-owned).
 *   n: at most 524288 (2^19) rays per call, else RTMC_EINVAL; larger sets
 *      are traced in several calls.
 *   The BVH's global traversal stack lives in the same array, so fewer
 *   persistent workgroups may be launched than the launch shape asks for;
 *   a tree too deep for it is refused with RTMC_EINVAL.
 *   Every call on one GPU uses that GPU's one array: calls whose work
 *   overlaps on the device (other streams, other contexts, other host
 *   threads) race and give wrong results; calls on one stream are ordered
 *   and safe. */
rtmc_status rtmc_first_hit_noalloc(rtmc_ctx* ctx, int32_t scene_id, const float* rays, int64_t n,
                                   int32_t* tri_out, float* t_out);

/* In-place ascending sort of (key, value) pairs by the low key_bits bits of
 * the keys (device radix sort used by the BVH builder; stable).
 *   keys: device uint64 [n]; vals: device uint32 [n]; 1 <= key_bits <= 64.
 *   Asynchronous on the context stream. */
rtmc_status rtmc_sort_pairs_u64(rtmc_ctx* ctx, uint64_t* keys, uint32_t* vals, int64_t n, int32_t key_bits);

rtmc_status rtmc_set_launch(rtmc_ctx* ctx, const rtmc_launch_cfg* cfg);
rtmc_status rtmc_get_launch(rtmc_ctx* ctx, rtmc_launch_cfg* cfg);

/* Time launch shapes on a calibration trace of the scene (n_primaries at
 * E_eV, theta_deg) and keep the fastest, also returned in *best.  Coordinate
 * search over block size, workgroups per compute unit, LDS stack depth,
 * refill threshold, kernel build (waves per SIMD), rays per wave per claim
 * and primaries per chunk (a half, quarter or eighth of n_primaries, else the
 * current chunk, which the calibration trace cannot tell from any other of at
 * least its length); a change is kept only if it is more than 2 % faster.
 * The winner is cached for the process, keyed by the GPU
 * (architecture, compute units), the scene's size (triangles as a power of
 * two, BVH depth), the tables' largest yield and the calibration point: a
 * call with the same key takes the cached shape without timing. */
rtmc_status rtmc_autotune(rtmc_ctx* ctx, int32_t scene_id, int32_t table_id, double E_eV, double theta_deg,
                          uint64_t n_primaries, rtmc_launch_cfg* best);

/* Streaming device copy of `bytes` bytes, repeated `reps` times; *ms is the
 * mean time per copy (the achievable-bandwidth probe). */
rtmc_status rtmc_copy_probe(rtmc_ctx* ctx, void* dst, const void* src, size_t bytes, int32_t reps, double* ms);

/* ---- Learned surrogate of the yield (an extension of the method: trained on
 * yields that rtmc_trace produces; plain RTMC stays the reference).
 * Architecture: n_in inputs -> depth hidden layers of width GELU units -> 1
 * output; BF16 operands on the matrix cores with FP32 accumulation; FP32
 * master weights updated with AdamW.  Only width 256 and depth 4 are built.
 * GELU(z) = z Phi(z), evaluated as max(z, 0) - |z| Phi(-|z|) with the normal
 * tail from the erfc of Abramowitz-Stegun 7.1.26 (absolute error <= 2.1e-7).
 * Parameter vector order (FP32): W1 [width x n_in] (row = output unit), b1
 * [width], W2 [width x width], b2, ..., W_depth, b_depth, w_out [width],
 * b_out [1]; rtmc_srg_param_count gives its length.
 * X: device float [n, n_in] (features already normalised by the caller);
 * y: device float [n].  Training and gradient calls need batch % 32 == 0
 * (at most 2^22 rows); they run in passes of at most 16384 rows (forward and
 * backward signals of 32-row tiles, then the weight gradients as GEMMs over
 * the pass's rows), then the update; every sum has a fixed order, so
 * gradients and training are reproducible bit for bit.
 * ENOTIMPL when the device offers less than 122 KB of LDS per workgroup. */
rtmc_status rtmc_srg_create(rtmc_ctx* ctx, int32_t n_in, int32_t width, int32_t depth, uint64_t seed,
                            int32_t* srg_id); /* 1 <= n_in <= 32; He-uniform weights, zero biases */
rtmc_status rtmc_srg_param_count(rtmc_ctx* ctx, int32_t srg_id, int64_t* n);
rtmc_status rtmc_srg_get_params(rtmc_ctx* ctx, int32_t srg_id, float* params, int64_t n); /* host */
rtmc_status rtmc_srg_set_params(rtmc_ctx* ctx, int32_t srg_id, const float* params, int64_t n); /* host; resets AdamW */
/* Mean-squared-error loss and its gradient (host float [n params], may be NULL) without an update. */
rtmc_status rtmc_srg_gradient(rtmc_ctx* ctx, int32_t srg_id, const float* X, const float* y, int64_t batch,
                              float* loss, float* grads);
/* One AdamW step (beta 0.9 / 0.999, eps 1e-8) on a batch; *loss is the batch loss before the step. */
rtmc_status rtmc_srg_train_step(rtmc_ctx* ctx, int32_t srg_id, const float* X, const float* y, int64_t batch,
                                float lr, float weight_decay, float* loss);
/* A training loop in one call: `steps` AdamW steps (as rtmc_srg_train_step),
 * step s on a batch of `batch` rows drawn on the device from the n rows of
 * (X, y), uniformly with replacement (Philox4x32-10, key seed, counter
 * (row, s, 0, 0)), at learning rate lr[s] (host float [steps]).
 * use_graph != 0: one step is captured as a HIP graph (again whenever the
 * arrays, sizes, seed or weight decay change) and replayed `steps` times,
 * so the loop runs without host round trips; 0: the same launches issued one
 * by one (identical results).  losses: host float [steps] (each step's batch
 * loss before its update), may be NULL.  X: device [n, n_in]; y: device [n];
 * n < 2^32; batch % 32 == 0.  Synchronous. */
rtmc_status rtmc_srg_train(rtmc_ctx* ctx, int32_t srg_id, const float* X, const float* y, int64_t n, int64_t batch,
                           int32_t steps, const float* lr, float weight_decay, uint64_t seed, int32_t use_graph,
                           float* losses);
/* Predictions for n rows (any n), written to device float y[n]; asynchronous on the context stream.
 * One fused kernel per call: each workgroup runs all layers for 128 rows with
 * the activations held in LDS (BF16 between layers), so the call allocates
 * nothing and touches memory only for X, y and the weights. */
rtmc_status rtmc_srg_predict(rtmc_ctx* ctx, int32_t srg_id, const float* X, int64_t n, float* y);

#ifdef __cplusplus
}
#endif
#endif /* RTMC_H */
