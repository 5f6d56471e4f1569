// Internal declarations shared by the host setup, the C ABI and the kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <complex>
#include <string>
#include <vector>

#include "../../include/abc_dtn.h"

namespace abc {

using cd = std::complex<double>;

constexpr int kMaxR = 3;

// Geometry of the box and of its six face slabs.  Face f = 2*axis + side,
// axis 0 = x, 1 = y, 2 = z; side 0 = low, 1 = high.  Transverse coordinates
// (t_slow, t_fast) are (z, y) for x-faces, (z, x) for y-faces, (y, x) for
// z-faces; layer 0 is the outermost box layer.
struct Geometry {
  int nx, ny, nz, R, batch;
  long long npts;            // nx*ny*nz
  long long face_off[7];     // element offsets of each face slab (units of complex * batch)
  int face_n1[6], face_n2[6];
};

Geometry make_geometry(int nx, int ny, int nz, int R, int batch);

// Box-form operator shapes for n = n_Gamma.  Boundary variables per orbital:
// none (zeroth), f (first) or f, g (second, Sec. 3.3).  The row-major
// operator is M (n x n), [B | A] (n x 2n) or [[0, I, A1], [B0, B1, C]]
// (2n x 3n): rows = the boundary variables' derivatives (or M E psi),
// columns = [boundary variables; E psi].
inline int box_aux_rows(int order, int n) { return order == ABC_SECOND ? 2 * n : (order == ABC_FIRST ? n : 0); }
inline int box_rows(int order, int n) { return order == ABC_ZEROTH ? n : box_aux_rows(order, n); }
inline int box_cols(int order, int n) { return box_aux_rows(order, n) + n; }
inline size_t box_mat_elems(int order, int n) { return (size_t)box_rows(order, n) * box_cols(order, n); }

// Host setup products ------------------------------------------------------

// Central second-derivative weights c_0..c_R.
void fd_weights(int R, double* c);

struct FaceOps {
  int R = 1, w = 0;
  std::vector<cd> kernel;    // [l][l'][p1+w][p2+w]
  cd a[kMaxR * kMaxR];       // normal-line block of A (first order)
  cd q[kMaxR * kMaxR];       // Lyapunov weight (H_gs H_gs^T)^{-1}
  double kernel_abs_sum = 0; // max over l of sum_{l',p} |k| (spectral bound)
  double symbol_norm = 0;    // sup over modes of the Frobenius norm of the
                             // (Lyapunov-weighted) symbol
  double coupling_norm = 0;  // Frobenius norm of the face coupling block
};

// Half-line DtN symbol per transverse mode by cyclic reduction of the
// semi-infinite block-tridiagonal exterior operator (R x R result).
void halfline_symbol(int R, double h, cd shift, cd* out);

// Face operators; returns ABC_OK or ABC_EUNSTABLE (sign condition violated).
abc_status build_face_ops(const abc_params& p, FaceOps& ops, std::string& err);

// Box form: dense operators built on the device.  mat_dev receives the
// row-major operator (box_rows x box_cols), q_dev the first order's
// Lyapunov weight (n x n) or NULL, subspace_dim the dimension of the
// subspace the second order interpolates in (n_Gamma otherwise).
// Second order in a subspace of dimension r < n_Gamma: the orthonormal basis
// U (real, n_Gamma x r, column-major; Ut the same matrix row-major) and the
// reduced operator [[0, I, A1~], [B0~, B1~, C~]] (2r x 3r, row-major), device
// buffers owned by the caller (null, r = 0, when the second order uses no
// subspace).
struct BoxReduced {
  double* U = nullptr;
  double* Ut = nullptr;
  double2* red = nullptr;
  int r = 0;
};
abc_status build_box_ops(const abc_params& p, double2** mat_dev, double2** q_dev, int* n_gamma,
                         std::vector<int>& gamma_lin, double* spectral_bound, int* subspace_dim, BoxReduced* reduced,
                         std::string& err);

}  // namespace abc

// Kernel launchers (kernels.hip) -------------------------------------------

// Long-range mean-field potentials (poisson.hip): conjugate-gradient state
// and work buffers over the box, all FP64 device memory except `host`
struct PotentialSolver {
  int nx = 0, ny = 0, nz = 0, R = 1;
  double h = 0, c[abc::kMaxR + 1] = {0, 0, 0, 0};
  double v0 = 0, a = 1, e2 = 0, tol = 1e-12;
  int maxit = 1000, nblk = 0;
  double *rho = nullptr, *wy = nullptr, *wc = nullptr;  // density, Yukawa and Coulomb fields (persist)
  double *r = nullptr, *p = nullptr, *q = nullptr;      // CG vectors
  double *part = nullptr, *scal = nullptr;              // 3 nblk partial sums, scalar slots
  double* host = nullptr;                               // pinned: convergence flag, iteration count
  int fixed = 0;                                        // > 0: iterations per solve, no host reads
  double* tally = nullptr;                              // device: Yukawa, Coulomb iterations, unconverged solves
  // sine-transform preconditioner: DST-I matrices and R = 1 eigenvalues per
  // axis, its work vectors, the preconditioned residual and a rocBLAS handle
  double *sx = nullptr, *sy = nullptr, *sz = nullptr, *ex = nullptr, *ey = nullptr, *ez = nullptr;
  double *t1 = nullptr, *t2 = nullptr, *z = nullptr;
  void* blas = nullptr;
  long long iters_y = 0, iters_c = 0, solves = 0;
};

// Exact face sections (fejer = 0, window >= max(n) - 1) applied by FFT:
// every face layer zero-padded to P1 x P2 (powers of two >= 2 n - 1), the
// kernel's spectra precomputed per face pair (x, y, z faces share sizes and
// kernel), circular convolution in the transform domain (kernels_staged.hip)
struct FaceFFT {
  int P1[3], P2[3], S[3];      // per face pair: padded sizes, slabs (2 faces x R layers x batch)
  long long woff[4];           // each pair's slabs in W and Z (complex elements)
  long long soff[4];           // each pair's R x R kernel spectra in spec
  long long twoff[3][4];       // twiddles per pair: forward / inverse along t2, forward / inverse along t1
  int lg1[3], lg2[3];          // log2 P1, log2 P2
  int twr[3], twc[3];          // lines per workgroup: row passes (along t2), column pass (along t1, R layers)
  int stwr[3], stwc[3];        // 1: those passes keep their twiddle table in LDS
  double2 *W, *Z, *spec, *tw;
};

// Boundary-shell buffers of the one-pass sweep with a non-local face
// operator: four psi-sized arrays (only their shell points are used) and two
// face-aux arrays.
struct ShellScratch {
  void* vol[4];
  double2* face[2];
};

struct abc_launch {
  abc::Geometry g;
  double h, dt;
  double c[abc::kMaxR + 1];
  int order, form, periodic, dtype, w;
  int meanfield;
  double t0, t3;
  PotentialSolver* pot;        // ABC_MF_SKYRME solves (or null)
  // face operators
  const double2* face_ker;
  const FaceFFT* face_fft;     // exact sections by FFT (staged path), or null
  double2 a_loc[abc::kMaxR * abc::kMaxR];
  double2 q_loc[abc::kMaxR * abc::kMaxR];
  double2 fused_m0, fused_b0;  // window-0 face operator value (host copy)
  // one-pass sweep: the step polynomial as (1 + a1 x + b1 x^2)(1 + a2 x + b2 x^2)
  double fused_a1, fused_b1, fused_a2, fused_b2;
  int fused_stages;            // 4: one launch per step; 2: two launches
  int fused_shell;             // one-pass sweep plus boundary-shell rounds (first order, window > 0)
  ShellScratch shell;
  int fused_tz;                // planes per tile of the two-stage kernel (4, 8, 16)
  // box form
  const double2* box_mat;
  const double2* box_q;       // Lyapunov weight (H_gs H_gs^T)^{-1}, n x n
  // second order in a subspace (box_r > 0): U (column-major, the
  // projection; Ut row-major, the lift) and the reduced operator; one
  // orbital steps through them instead of box_mat
  const double* box_U;
  const double* box_Ut;
  const double2* box_red;
  int box_r;
  const int* gamma_lin;       // gamma index -> linear point index
  const int* point_gamma;     // linear point index -> gamma index or -1
  int n_gamma;
};

struct abc_scratch {
  void* y[2];          // stage vectors (psi dtype)
  void* acc;           // Taylor accumulator (psi dtype)
  double2* g[2];       // aux stage vectors
  double2* facc;       // aux accumulator
  double2* src;        // zeroth-order source on the faces / Gamma
  void* veff;          // V + mean field (psi real dtype)
  double* red;         // reduction partials
  int red_blocks;
  double2* bwork[2];   // box form over a batch: gathered E y, GEMM result ([gamma][orbital])
  double2* bpart;      // box form over a batch: partial GEMM results when K is split over workgroups
  double* bpack;       // second order in a subspace: 6 x n_Gamma packed vectors
  double* bred;        // second order in a subspace: 20 r doubles of reduced vectors
};

// Per-launch timing for measurement runs: every kernel launch of a step is
// issued through hipExtLaunchKernel with a fresh start/stop event pair, so
// the pair brackets exactly that kernel's execution.  The first step's labels
// name the launches of a step.
struct abc_timer {
  struct span { hipEvent_t start, stop; };
  std::vector<span> ev;
  std::vector<std::string> labels;
  int steps_done = 0;
  hipError_t err = hipSuccess;
  bool pair(const char* label, hipEvent_t* start, hipEvent_t* stop) {
    hipError_t r = hipEventCreate(start);
    if (r == hipSuccess) {
      r = hipEventCreate(stop);
      if (r != hipSuccess) hipEventDestroy(*start);
    }
    if (r != hipSuccess) {
      if (err == hipSuccess) err = r;
      return false;
    }
    ev.push_back({*start, *stop});
    if (steps_done == 0) labels.emplace_back(label);
    return true;
  }
  // a library call (rocBLAS) inside a step is not timed; it is named so that
  // the labels still describe the timed launches
  void mark_host(hipStream_t, const char*) {}
  void end_step() { ++steps_done; }
  ~abc_timer() {
    for (span& s : ev) {
      hipEventDestroy(s.start);
      hipEventDestroy(s.stop);
    }
  }
};

// Launches kernel k; with a timer, through hipExtLaunchKernel with a start and
// stop event recorded around it.
template <typename... P, typename... A>
void abc_launch_kernel(abc_timer* tm, const char* label, void (*k)(P...), dim3 grid, dim3 block, hipStream_t st,
                       A... args) {
  if (!tm) {
    k<<<grid, block, 0, st>>>(args...);
    return;
  }
  hipEvent_t e0, e1;
  if (tm->pair(label, &e0, &e1)) hipExtLaunchKernelGGL(k, grid, block, 0, st, e0, e1, 0, args...);
}

// the same with `lds` bytes of dynamic LDS
template <typename... P, typename... A>
void abc_launch_kernel_lds(abc_timer* tm, const char* label, void (*k)(P...), dim3 grid, dim3 block, size_t lds,
                           hipStream_t st, A... args) {
  if (!tm) {
    k<<<grid, block, lds, st>>>(args...);
    return;
  }
  hipEvent_t e0, e1;
  if (tm->pair(label, &e0, &e1)) hipExtLaunchKernelGGL(k, grid, block, lds, st, e0, e1, 0, args...);
}

// keep (optional): three psi-sized buffers that receive the stage vectors
// z_1, z_2, z_3 of the (last) step instead of the scratch ping-pong.
// psi_in, aux_in (optional): the first step reads its state from these
// instead of psi and aux, which receive the result; the inputs are left as
// they were (a step out of place, without a copy).
// elements of abc_scratch::bpart for a box-form orbital batch whose GEMM
// result has `result_elems` elements (rows x orbitals)
size_t box_gemm_part_elems(size_t result_elems);

hipError_t launch_step_staged(const abc_launch& L, const abc_scratch& S, void* psi, double2* aux,
                              const void* V, int n_steps, hipStream_t st, abc_timer* tm = nullptr,
                              void* const* keep = nullptr, const void* psi_in = nullptr,
                              const double2* aux_in = nullptr);
// One fused step out of place (psi_in, aux_in) -> (psi_out, aux_out) on the
// two-stage kernels (L must satisfy fused_supported), keeping the Horner
// intermediates u1, u2, u3 of the step in keep[0..2] (psi-sized).
hipError_t launch_step_fused_keep(const abc_launch& L, const abc_scratch& S, const void* psi_in,
                                  const double2* aux_in, void* psi_out, double2* aux_out, const void* V,
                                  void* const* keep, hipStream_t st);
// The same (complex128) keeping the increments u1 - z, u2 - z, u3 - z of the
// intermediates over the step's input z in keep[0..2] (differences without
// cancellation); uses S.y[1] for u2.
hipError_t launch_step_fused_keepd(const abc_launch& L, const abc_scratch& S, const void* psi_in,
                                   const double2* aux_in, void* psi_out, double2* aux_out, const void* V,
                                   void* const* keep, hipStream_t st);
// Discrete adjoint (adjoint.hip).  La is L with the adjoint operators
// (dt -> -dt, conjugate-transposed boundary operators, rescaled aux).
struct abc_adjoint_args {
  const void* psi0;
  const void* V;
  int n_steps, stride, objective;
  void* grad_psi0;
  double* grad_V;
  double* J_host;
  int use_fused;  // forward sweep on the fused path
};
// Build the FFT plan of the exact face sections (device buffers appended to
// allocs); the kernel is ops.kernel, of width w >= max(n) - 1
abc_status face_fft_setup(const abc::Geometry& g, int R, int w, const std::vector<abc::cd>& kernel, FaceFFT& ff,
                          std::vector<void*>* allocs, size_t* bytes, std::string& err);

// V + t0 rho + t3 rho^2 + W_Y + W_C for psi ([point][orbital], or orbital
// arrays when soa) into veff; synchronises the stream during the solves
hipError_t potential_warmup(PotentialSolver& ps);
hipError_t skyrme_veff(PotentialSolver& ps, const void* psi, bool soa, int B, bool c64, const void* V, void* veff,
                       double t0, double t3, hipStream_t st, abc_timer* tm);

// H2 objective of candidate first-order points (face form, R = 1): out[c]
// for s1[c]; synchronises the stream (h2.hip)
abc_status run_h2_objective(const abc_params& p, const double* s1, int count, int modes, int nodes, double* out,
                            hipStream_t st, std::string& err);

abc_status run_adjoint(const abc_launch& L, const abc_launch& La, const abc_scratch& S, const abc_adjoint_args& a,
                       hipStream_t st, std::string& err);

// Reduction partials go to red, or to the context's S.red when red is null.
hipError_t launch_diagnostics(const abc_launch& L, const abc_scratch& S, const void* psi,
                              const double2* aux, const void* V, double* out, hipStream_t st,
                              double* red = nullptr);

// Boundary-shell rounds of the one-pass sweep (first order, face form with a
// non-local operator, R = 1, one orbital): from the step's input (psi, f)
// they write the new aux to fout and add the boundary's correction to
// psi_out, the condition-free sweep of the same input.
hipError_t launch_shell_rounds(const abc_launch& L, const ShellScratch& W, const void* psi, const void* V,
                               const double2* f, double2* fout, void* psi_out, hipStream_t st, abc_timer* tm);

// Doubles of reduction partials one diagnostics call writes for a batch.
size_t diag_partial_doubles(int batch);

// One-block check of a monitor record (abc_step_monitored): writes the step
// count to rec[0] and ors the ABC_FLAG_* conditions of rec[1..] into *flags.
hipError_t launch_monitor_check(double* rec, int batch, long long step, double* prevW, bool have_prev, bool check_w,
                                double tol, unsigned* flags, hipStream_t st);
