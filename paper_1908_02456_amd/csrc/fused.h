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
