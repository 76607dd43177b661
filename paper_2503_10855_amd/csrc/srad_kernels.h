// srad_kernels.h -- host-side entry points of the SRAD sweeps (k_srad.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace hx {

// ---- SRAD ------------------------------------------------------------
// Workgroups of one SRAD launch over an H x W image (4 sweep items of 256
// columns x 32 rows each); the partial-sum buffer holds 4 doubles per
// workgroup (two halves of one pair each).
int64_t srad_blocks(int64_t H, int64_t W);
// niter iterations on J (pitch pj): iteration k reads one of J / Jb and
// writes the other, starting from J (so an odd niter ends in Jb).  cbuf
// (pitch pc) is the unfused form's c plane; q_log (nullable) receives
// niter doubles.
hipError_t launch_srad(const float* J, float* Jb, int64_t pj, int64_t pb, float* cbuf,
                       int64_t pc, double* partials, double* q_log, int H, int W,
                       int niter, float lambda, bool fused, hipStream_t s);

}  // namespace hx
