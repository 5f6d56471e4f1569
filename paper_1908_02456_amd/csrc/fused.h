// Fused single-pass Taylor-4 step (face form with a local boundary operator,
// Dirichlet and periodic boxes).  Declarations shared with the C ABI.
#pragma once

#include <string>
#include <vector>

#include "abc_internal.h"

// true when the fused kernel covers the parameters; otherwise *why says why
bool fused_supported(const abc_params& p, std::string* why);
// the same for the one-pass sweep (all four stages in one launch)
bool fused4_supported(const abc_params& p, std::string* why);
// first order in the face form with a non-local operator (window > 0): the
// one-pass sweep runs without the condition plus the boundary-shell rounds
bool fused_shell_case(const abc_params& p);

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

// Orbital batches (and the mean field) on the fused path: the orbitals are
// transposed once per call from [point][orbital] to one array per orbital,
// stepped as boxes of a descriptor-driven launch sharing one potential (the
// mean field rebuilt from the current state before every step), and
// transposed back.  All buffers below are owned by the context.
struct OrbitalBatch {
  abc_launch L1;                   // the launch of one orbital (batch 1 geometry)
  int B = 0;                       // orbitals
  int tz = 8;
  void* soa[3] = {nullptr, nullptr, nullptr};  // psi arrays [B][npts]: state A, state B, u2
  double2* soa_f[3] = {nullptr, nullptr, nullptr};  // aux arrays [B][nface]: A, B, aux of u2
  void* veff = nullptr;            // V + mean field (psi's real type), or null
  // descriptors of the two-stage launches, one set per step-count parity,
  // built on first use for a given potential buffer and reused after that
  // (so a warmed-up step issues no copy and can be captured in a graph)
  void* desc_host = nullptr;       // pinned staging, two sets
  void* desc_dev = nullptr;        // two sets
  const void* desc_V[2] = {nullptr, nullptr};
  bool desc_ok[2] = {false, false};
  int desc_total = 0;
  hipEvent_t copied = nullptr;
  bool pending = false;
  std::vector<abc_scratch> S;      // per-orbital scratch views into soa / soa_f
};
size_t orbital_batch_bytes(const abc_launch& L1, int B, bool first, bool meanfield);
hipError_t launch_step_orbitals(OrbitalBatch& ob, void* psi, double2* aux, const void* V, int n_steps,
                                hipStream_t st, abc_timer* tm);
