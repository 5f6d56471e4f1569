// Fused single-pass Taylor-4 step (face form with a local boundary operator,
// Dirichlet and periodic boxes).  Declarations shared with the C ABI.
#pragma once

#include <string>
#include <vector>

#include "abc_internal.h"

// true when the fused kernel covers the parameters; otherwise *why says why
bool fused_supported(const abc_params& p, std::string* why);

// allocate/prepare whatever the fused path needs beyond the staged scratch
abc_status fused_prepare(const abc_params& p, abc_launch& L, std::vector<void*>* allocs, size_t* bytes,
                         std::string& err);

hipError_t launch_step_fused(const abc_launch& L, const abc_scratch& S, void* psi, double2* aux, const void* V,
                             int n_steps, hipStream_t st, abc_timer* tm = nullptr);

// largest tile depth (planes) the two-stage kernel can use for this order/box
int fused_max_tz(int order, int nz);
bool fused_tz_valid(const abc_launch& L, int tz);

// Batched two-stage launch over boxes sharing (order, precision, tile depth).
// fused_batch_build writes 4 descriptor sets (step parity x half) for an
// n-step call into `host` (fused_batch_desc_bytes(nbox) bytes) and returns the
// total tile count; once they are in device memory at `dev`,
// launch_batch_fused runs the n steps as 2 launches per step over the
// concatenated tiles of all boxes.
struct FusedMember {
  const abc_launch* L;
  const abc_scratch* S;
  void* psi;
  double2* aux;
  const void* V;
};
size_t fused_batch_desc_bytes(int nbox);
int fused_batch_build(const std::vector<FusedMember>& m, void* host, int n);
hipError_t launch_batch_fused(const std::vector<FusedMember>& m, int tz, const void* dev, int total, int n,
                              hipStream_t st, abc_timer* tm);
