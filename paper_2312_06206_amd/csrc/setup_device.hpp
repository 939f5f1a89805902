// Batched set-up of the Gohberg-Semencul line tables (Proposition 1, Algorithm 1): the
// declarations shared by the context set-up, the batch and setup_device.hip.
#pragma once

#include <hip/hip_runtime.h>

namespace sadi {

// One context's tables: c = H_M^-1 e_1 from t = t_hi + t_lo (the first column of H_M, m <= 4096
// entries), then lam_s, lam_c, f and their float32 copies, as launch_gs_generator makes them.
struct GsJob {
  const double* t_hi;
  const double* t_lo;
  double* c;
  const double2* q;
  double2* lam_s;
  double2* lam_c;
  double* f;
  float2* lam_s32;
  float2* lam_c32;
  float* f32;
  int m;
};

// Many contexts at once (a batch's set-up): one Levinson workgroup per job in one launch, then
// the tables of every job in a second.  jobs: device array of njobs; max_m: the largest m.
void launch_gs_generator_batched(const GsJob* jobs, int njobs, int max_m, hipStream_t st);

}  // namespace sadi
