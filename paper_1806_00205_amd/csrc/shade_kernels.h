// Internal declarations of the shading kernel (shade.hip), used by the host
// runtime: the flat-surface tables as the kernel sees them, the argument
// block of one shading launch and its launchers.
#pragma once

#include "rtmc_internal.h"

namespace rtmc {

constexpr int32_t kEmitPaper = 1;  // DevTables::emission of the paper's one/two-daughter rule
constexpr int kGuide = 1024;       // entries of each CDF guide table
constexpr int kShadeJobs = 32;     // chunks with at most this many jobs tally per workgroup in LDS

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

// LDS of a shading workgroup; n_jobs = jobs of the chunk (tallied in LDS when <= kShadeJobs)
size_t shade_lds_bytes(const DevTables& tb, int n_hist, int block, int n_jobs);  // n_hist: all histogram bins
hipError_t launch_shade(const ShadeArgs& a, int n_cu, int block, hipStream_t s);  // grid = n_cu x occupancy
hipError_t launch_chunk_reduce(const DevJob* jobs, int32_t j_lo, int32_t j_hi, const uint32_t* ppc, uint32_t n,
                               uint64_t chunk_lo, hipStream_t s);

}  // namespace rtmc
