/*
 * abc_dtn.h -- C ABI of the gfx950 time stepper for the semi-discrete 3D
 * Schroedinger equation closed by discrete Dirichlet-to-Neumann absorbing
 * boundary conditions (Wu & Li, arXiv:1908.02456).
 *
 * What is computed
 * ----------------
 * The box holds nx*ny*nz grid points x_j = (j - (n-1)/2) h per axis.  Inside
 * it the Hamiltonian is H = -(1/2) Delta_h + V (hbar = m = 1, Sec. 2), with
 * Delta_h the axis-by-axis central difference of half-width R (R = 1 is the
 * 3D seven-point Laplacian; R = 3 is the paper's "seven points in each
 * direction").  The exterior (V = 0) acts on the box only through the
 * boundary layer Gamma (points within R of a face), Sec. 2.  The supported
 * dynamics are (Sec. 3):
 *   ABC_ZEROTH:  d/dt psi = -i (H psi + E^T M E psi),  M = K(s0)
 *   ABC_FIRST:   d/dt psi = -i H psi - i E^T f,  d/dt f = B f + A E psi,
 *                A = -i H_{Gamma,II} H_{II,Gamma},  B = s1 I - A K(s1)^{-1}
 *                (the first-order stability theorem), or with a finite s2 the
 *                two-point interpolation R11(s1) = K(s1), R11(s2) = K(s2)
 *   ABC_SECOND:  the second-order approximation of Sec. 3.3,
 *                K(s) ~ (s^2 I - s B1 - B0)^{-1} (s A1 + A0), interpolating
 *                K at the four points s1, s2, s3, s4; its dynamics
 *                d2f/dt2 = B1 df/dt + B0 f + A1 E dpsi/dt + A0 E psi run as
 *                the first-order system in (psi, f, g), g = df/dt - A1 E psi:
 *                d/dt psi = -i H psi - i E^T f,  d/dt f = g + A1 E psi,
 *                d/dt g = B1 g + B0 f + (B1 A1 + A0) E psi  (box form only;
 *                the paper gives no stability theorem for this order)
 *   ABC_DIRICHLET / ABC_PERIODIC: no condition (zero outside / wrap-around),
 * where K(s) is the discrete DtN map (Sec. 2, evaluated by the App. A
 * boundary-element formula).  Time stepping is the fourth-order Taylor
 * propagator of Sec. 4, sum_{k<=4} (dt L)^k / k!, applied to the generator L
 * of the (augmented) linear dynamics; with a mean field (Sec. 4.3, simplified
 * to U = t0 rho + t3 rho^2, rho = sum over the batch of |psi_j|^2) U is
 * rebuilt from the state at the start of every step.
 *
 * Two forms of the boundary operators:
 *   ABC_FORM_BOX    the paper's dense n_Gamma x n_Gamma matrices (exact;
 *                   memory n_Gamma^2 * 16 B, so only for small boxes).
 *   ABC_FORM_FACES  each face sees the half-space beyond it; its operator is
 *                   the Toeplitz section, over the face's R-layer slab, of the
 *                   half-space DtN kernel, truncated to |p|_inf <= window and
 *                   (fejer = 1) tapered by the separable triangular window,
 *                   which keeps both stability theorems' sign conditions.
 *                   window >= max(n)-1 with fejer = 0 is the exact section,
 *                   applied by zero-padded 2D FFTs (padded side P = the
 *                   power of two >= 2n - 1; ABC_ENOTSUP unless R * P <= 4096
 *                   on every face).
 *
 * Memory, layout and ownership
 * ----------------------------
 * All state buffers are device memory owned by the caller:
 *   psi  complex, [z][y][x][orb] (orbital fastest; x fastest when batch = 1),
 *        interleaved (re, im); complex128 for ABC_C128, complex64 for ABC_C64.
 *   V    real external potential [z][y][x], float64 (ABC_C128) or float32
 *        (ABC_C64); may be NULL for V = 0.
 *   aux  complex128 always (the auxiliary recurrences stay in FP64),
 *        abc_aux_elems() elements, zero at t = 0 (the exterior starts empty,
 *        Sec. 2).  Face form: [face][layer][t_slow][t_fast][orb] with faces in
 *        the order x-,x+,y-,y+,z-,z+; layer 0 is the outermost box layer;
 *        (t_slow, t_fast) = (z, y) for x-faces, (z, x) for y-faces, (y, x)
 *        for z-faces.  Box form: [gamma][orb], Gamma in C order of (z, y, x);
 *        second order holds f then g, each [gamma][orb].
 * The context owns only setup products (operators) and scratch.
 *
 * Errors and threading
 * --------------------
 * Every call returns an abc_status; no exception crosses the ABI.  The text
 * of the last error of the calling thread is returned by abc_last_error().
 * All device work of abc_step/abc_diagnostics is queued on the given stream
 * (a hipStream_t passed as void*; NULL = the default stream) and nothing
 * synchronises with the host.  One context must not be used by two streams
 * at once (it owns the scratch buffers).
 */
#ifndef ABC_DTN_H
#define ABC_DTN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct abc_ctx abc_ctx;

typedef enum {
  ABC_OK = 0,
  ABC_EINVAL = -1,     /* invalid parameters or buffer sizes               */
  ABC_ENOMEM = -2,     /* device or host allocation failed                 */
  ABC_EDEVICE = -3,    /* a HIP runtime or library call failed             */
  ABC_EUNSTABLE = -4,  /* stability self-check at setup failed             */
  ABC_ENOTSUP = -5,    /* combination not implemented                      */
  ABC_EIO = -6         /* a checkpoint file could not be read or written   */
} abc_status;

enum { ABC_DIRICHLET = 0, ABC_PERIODIC = 1, ABC_ZEROTH = 2, ABC_FIRST = 3, ABC_SECOND = 4 };
enum { ABC_FORM_BOX = 0, ABC_FORM_FACES = 1 };
enum { ABC_C128 = 0, ABC_C64 = 1 };
enum { ABC_MF_NONE = 0, ABC_MF_T0T3 = 1, ABC_MF_SKYRME = 2 };
/* execution path of abc_step */
enum { ABC_PATH_AUTO = 0, ABC_PATH_STAGED = 1, ABC_PATH_FUSED = 2, ABC_PATH_ONEPASS = 3 };

typedef struct {
  int nx, ny, nz;     /* box points per axis (>= 2R + 1)                     */
  double h, dt;       /* grid spacing, time step                            */
  int radius;         /* R in {1, 2, 3}                                     */
  int order;          /* ABC_DIRICHLET | ABC_PERIODIC | ABC_ZEROTH | ABC_FIRST
                         | ABC_SECOND                                        */
  int form;           /* ABC_FORM_BOX | ABC_FORM_FACES                      */
  double s0;          /* zeroth-order interpolation point (> 0)             */
  double s1, s2;      /* first-order points; s2 <= 0 selects the theorem's
                         (s1, infinity) pair; s2 > 0 two-point (box form).
                         Second order: the first two of its four points     */
  int window;         /* face form: kernel half-width w (|p|_inf <= w)       */
  int fejer;          /* face form: 1 = triangular window, 0 = truncation    */
  int dtype;          /* ABC_C128 | ABC_C64                                 */
  int batch;          /* wavefunctions sharing grid, V and boundary (>= 1)  */
  int meanfield;      /* ABC_MF_NONE | ABC_MF_T0T3                          */
  double t0, t3;      /* mean-field coefficients                            */
  int path;           /* ABC_PATH_AUTO: the one-pass sweep (all four stages
                         in one launch per step) where it covers the
                         parameters (for the first order only on rows of
                         128 columns), else the two-stage fused kernels,
                         else the staged path.  ABC_PATH_FUSED / ABC_PATH_ONEPASS
                         force those kernels (ABC_ENOTSUP when they do not
                         cover the parameters): R = 1, window 0, nx, ny >= 4,
                         nz >= 5; the one-pass sweep also one orbital, no
                         mean field, nx <= 128 and, for the first order,
                         ny > 12 / 16 and nz > 20 / 12 (complex128 /
                         complex64); ABC_PATH_STAGED the general path     */
  int diag_every;     /* abc_step_monitored: steps between diagnostic records
                         (>= 1 to monitor; 0 = no monitoring)               */
  int reserved[2];    /* must be zero                                       */
  double s3, s4;      /* second order: the last two interpolation points;
                         s1..s4 positive and distinct                       */
  /* ABC_MF_SKYRME (Sec. 4.3): U = t0 rho + t3 rho^2 + W_Y + W_C with
     (Delta_h - 1/a^2) W_Y = -4 pi v0 a rho and Delta_h W_C = -2 pi e2 rho on
     the box (Delta_h the wavefunctions' Laplacian, zero outside), solved by
     preconditioned conjugate gradients at the start of every step          */
  double v0, a_yukawa;  /* Yukawa strength and range (a > 0 unless v0 = 0) */
  double e2;            /* Coulomb e^2 (0: no Coulomb term)                 */
  double pcg_tol;       /* relative residual of the solves (> 0)            */
  int pcg_maxit;        /* iteration cap per solve (>= 1)                   */
  int pcg_fixed;        /* 0: each solve reads its convergence flag on the
                           host after every iteration and stops there (the
                           step synchronises its stream); k >= 1: each solve
                           issues exactly k iterations and reads nothing on
                           the host (iterations after convergence are
                           skipped on the device), so that abc_step can be
                           captured in a HIP graph; solves still unconverged
                           after k iterations are counted on the device
                           (abc_potential_unconverged)                     */
  int reserved2[2];     /* must be zero                                     */
} abc_params;

/* Fill p with defaults (R = 1, first order, face form, w = 0, fejer = 1,
 * s0 = s1 = 1, s2 = 0, s3 = 3, s4 = 10, C128, batch 1, no mean field,
 * automatic path; v0 = e2 = 0, a_yukawa = 1, pcg_tol = 1e-12,
 * pcg_maxit = 1000). */
void abc_params_default(abc_params* p);

/* Build the operators for p on the current HIP device (host FP64 setup;
 * may take seconds for the box form) and allocate the context's scratch.
 * Box form: K(s) by App. A, dense solves on the device.  Face form:
 * half-line DtN symbols per transverse mode, kernel coefficients.
 * Second order: box form only (ABC_ENOTSUP for the face form), the four
 * points positive and pairwise distinct (ABC_EINVAL otherwise); its
 * coefficients come from one square solve of the interpolation conditions
 * (Sec. 3.3).  For R >= 2 the four maps are numerically rank-deficient and
 * that system is singular in FP64, so the solve runs in the maps' dominant
 * subspace U (singular values of the four maps together above 1e-2 of the
 * largest; at R = 2 and 3 the boundary's outermost layer): the reduced maps
 * U^T K U are interpolated and the coefficients lifted as U X U^T, a
 * 4 r square solve (r = n_Gamma when nothing is dropped, as at R = 1).
 * Returns ABC_EUNSTABLE when a sign condition of the stability theorems
 * fails on the symbol, or when dt times the spectral-radius bound of the
 * kinetic and boundary operators exceeds the Taylor-4 stability limit
 * 2 sqrt(2) (for the second order the boundary part of that bound is a
 * power-iteration estimate of the spectral radius of the (f, g) block).
 * On success *out owns device memory until abc_destroy. */
abc_status abc_setup(const abc_params* p, abc_ctx** out);

/* Advance (psi, aux) by n_steps Taylor-4 steps in place.  psi, V, aux as
 * described above (aux may be NULL unless order is ABC_FIRST or ABC_SECOND).
 * No allocation, no host synchronisation, except with ABC_MF_SKYRME, whose
 * potential solves read their convergence flag on the host every 8
 * iterations. */
abc_status abc_step(abc_ctx* ctx, void* psi, void* aux, const void* V,
                    int n_steps, void* stream);

/* Flags of abc_step_monitored. */
enum { ABC_FLAG_NONFINITE = 1, ABC_FLAG_W_INCREASE = 2 };

/* abc_step with in-step monitoring (Sec. 3: the zeroth- and first-order
 * stability proofs make the Lyapunov functional W non-increasing).  After
 * every p.diag_every-th step counted over the context's monitored calls,
 * the norm, W and the energy of the state (the abc_diagnostics output,
 * 3*batch + 1 doubles) go to the device ring `ring` as one record of
 * 3*batch + 2 doubles: the step count, then that output; the k-th record
 * since setup goes to slot k mod ring_len.  The device word `flags`
 * (caller-owned, zero it to start) collects, by atomic or:
 *   ABC_FLAG_NONFINITE   a record holds a NaN or infinity (a blown-up or
 *                        corrupted state);
 *   ABC_FLAG_W_INCREASE  W of some orbital grew by more than 1e-12 of its
 *                        value since the previous record (zeroth and first
 *                        order, Dirichlet and periodic boxes; the second
 *                        order has no such functional and is not checked).
 * The host reads flags and the ring when it wishes (after synchronising the
 * stream); nothing here synchronises.  The records are separate reduction
 * launches on diagnostic steps only (the energy needs H of the new state,
 * which the sweeps do not form), using the context's reduction scratch:
 * one monitored call per context at a time.  ABC_EINVAL if p.diag_every
 * < 1, ring_len < 1 or a pointer is null. */
abc_status abc_step_monitored(abc_ctx* ctx, void* psi, void* aux, const void* V,
                              int n_steps, void* stream, double* ring, int ring_len,
                              unsigned* flags);

/* Measurement run: advances the state by n_steps (>= 1) exactly as abc_step
 * does, but issues every kernel launch through hipExtLaunchKernel with a
 * start/stop HIP event pair that brackets that kernel's execution, then
 * waits for the stream.  *launches receives the number k of kernel launches
 * per step; ms[j], for j < min(cap, k), the mean over the steps of the
 * duration in milliseconds of the j-th launch of a step.  abc_launch_label
 * names the launches.  Synchronises with the host; creates and destroys
 * 2 k n_steps events.  ABC_EINVAL on null arguments or n_steps < 1,
 * ABC_EDEVICE if a launch or an event call fails. */
abc_status abc_step_timed(abc_ctx* ctx, void* psi, void* aux, const void* V,
                          int n_steps, void* stream, double* ms, int cap,
                          int* launches);

/* Name of the j-th kernel launch of a step as timed by the last
 * abc_step_timed on ctx (owned by ctx, valid until the next such call or
 * abc_destroy); NULL if j is out of range or no timed call was made. */
const char* abc_launch_label(const abc_ctx* ctx, int j);

/* Objectives of abc_adjoint. */
enum { ABC_OBJ_PROB = 0, ABC_OBJ_ENERGY = 1 };

/* Discrete adjoint (reverse mode) of n_steps Taylor steps of the stepping map
 * of Sec. 4 on the dynamics of Sec. 3, started from (psi0, f = 0).
 * objective ABC_OBJ_PROB: J = h^3 sum |psi_N|^2 (probability left in the
 * box); ABC_OBJ_ENERGY: J = h^3 Re <psi_N, H_{I,I} psi_N> (no boundary term).
 * Writes J to the host double *J_out, dJ/dRe psi0 + i dJ/dIm psi0 to
 * grad_psi0 (device, complex128, psi's layout, caller-owned) and dJ/dV to
 * grad_V (device, float64 [z][y][x], caller-owned).  psi0 and V are device
 * buffers of the context's box (V may be NULL for V = 0).  Checkpoints every
 * ckpt_stride steps (<= 0: ceil(sqrt(n_steps))) during a forward sweep on
 * the context's path; each segment is recomputed once, keeping its states
 * and stage vectors.  Device memory for about n/stride + 4 stride + 8 states
 * is allocated and freed by the call, which synchronises the stream.  Supported: complex128, one orbital, no mean
 * field; Dirichlet and periodic boxes; face-form zeroth order (any R) and
 * first order (R = 1).  Others (the box form, the second order): ABC_ENOTSUP.  ABC_ENOMEM if the buffers do
 * not fit, ABC_EDEVICE on HIP failures. */
abc_status abc_adjoint(abc_ctx* ctx, const void* psi0, const void* V,
                       int n_steps, int ckpt_stride, int objective,
                       void* grad_psi0, double* grad_V, double* J_out,
                       void* stream);

/* Tile-depth tuner for the fused path: times a few steps with each tile depth
 * (4, 8 or 16 z-planes per tile, as the box and order allow) on the given
 * buffers and keeps the fastest for later abc_step calls; *tz_out (may be
 * NULL) receives it (0 on the staged path, which has nothing to tune).  The
 * state is restored afterwards; the call allocates temporary copies of psi
 * and aux and synchronises the stream. */
abc_status abc_tune(abc_ctx* ctx, void* psi, void* aux, const void* V,
                    void* stream, int* tz_out);

/* Batches of independent boxes (uneven sizes, mixed orders and precisions).
 * abc_setup_batch sets up n instances from ps[0..n-1] (each as abc_setup).
 * Instances that run on the fused path are grouped by (order, precision);
 * every group is stepped by one descriptor-driven launch per half step over
 * the concatenated tiles of all its boxes, with one tile depth per group
 * (abc_tune_batch picks it by timing).  Other instances are stepped one by
 * one with abc_step.  abc_step_batch advances instance i's psi[i] (and
 * aux[i], first and second order; V[i] may be NULL, V itself may be NULL for V = 0) by
 * n_steps on the stream; with ABC_BATCH_GRAPH in flags the whole call is
 * captured once into a HIP graph per (buffers, n_steps, stream), which later
 * calls with the same arguments replay (the stream must not be the default
 * stream).  Descriptor uploads are staged in pinned host memory; a call may
 * wait for the previous call's upload to complete.  Errors as abc_setup /
 * abc_step; setup errors name the instance. */
typedef struct abc_batch abc_batch;
enum { ABC_BATCH_GRAPH = 1 };
abc_status abc_setup_batch(const abc_params* ps, int n, abc_batch** out);
abc_status abc_step_batch(abc_batch* b, void* const* psi, void* const* aux,
                          const void* const* V, int n_steps, int flags,
                          void* stream);
abc_status abc_tune_batch(abc_batch* b, void* const* psi, void* const* aux,
                          const void* const* V, void* stream);
/* aux elements of instance i (as abc_aux_elems), 0 if out of range */
size_t abc_batch_aux_elems(const abc_batch* b, int i);
/* number of descriptor-driven launch groups, and the tile depth of one */
int abc_batch_launch_groups(const abc_batch* b);
int abc_batch_tile_depth(const abc_batch* b, int group);
void abc_destroy_batch(abc_batch* b);

/* H2 objective of the first-order interpolation point (Sec. 5 proposes the
 * minimiser of ||K(s) - R11(s)||_H2 as the best point).  For the face form
 * with R = 1 it is evaluated per half-space and per transverse Fourier mode:
 *   J(s1) = P^-2 sum_theta (1/2pi) int |k^(theta; i w) - a/(i w - b_w(theta))|^2 dw
 * with k^ the half-line DtN symbol on the imaginary axis (limit from
 * Re s > 0), a = -i H_gs H_gs^T and b_w the symbol of the kernel of B that
 * abc_setup builds at s1 with p's window and fejer settings (Theorem 3.2
 * per mode).  theta runs over the modes x modes grid 2 pi j / modes; the
 * frequency integral uses `nodes` midpoints of w = W0 (tan(phi) - 1),
 * W0 = 3/h^2.  p: a first-order face-form parameter set with radius 1
 * (its s1 is ignored); s1[0..count-1]: candidate points (host, > 0); out:
 * host array of count doubles.  Device memory is allocated and freed by the
 * call, which synchronises the stream.  ABC_EINVAL for bad sizes or points,
 * ABC_ENOTSUP for other orders, forms or radii, ABC_EUNSTABLE if the face
 * setup rejects a candidate. */
abc_status abc_h2_objective(const abc_params* p, const double* s1, int count,
                            int modes, int nodes, double* out, void* stream);

/* Effective potential V + U of the state psi for an ABC_MF_SKYRME context:
 * t0 rho + t3 rho^2 plus the Yukawa and Coulomb fields of rho = sum over
 * orbitals of |psi_j|^2, solved as in abc_step (the solves start from the
 * context's previous potentials).  psi, V (may be NULL) and out ([z][y][x],
 * the state's real type) are device buffers.  With pcg_fixed = 0 the call
 * synchronises the stream (the solves read their convergence flag on the
 * host).
 * ABC_ENOTSUP for other mean fields. */
abc_status abc_effective_potential(abc_ctx* ctx, const void* psi, const void* V,
                                   void* out, void* stream);

/* Conjugate-gradient work of the ABC_MF_SKYRME solves so far: out[0] =
 * number of mean-field evaluations, out[1] = Yukawa iterations, out[2] =
 * Coulomb iterations (all zero for other mean fields).  With pcg_fixed >= 1
 * the iteration counts are kept on the device and this call synchronises
 * the device to read them. */
abc_status abc_potential_iterations(const abc_ctx* ctx, long long* out);

/* Number of ABC_MF_SKYRME solves so far that ended without reaching
 * pcg_tol (at pcg_maxit, or after the pcg_fixed iterations), into *out;
 * counted on the device, so the call synchronises the device.  0 for other
 * mean fields. */
abc_status abc_potential_unconverged(const abc_ctx* ctx, long long* out);

/* FP64 diagnostics of a state, written to device memory out (3*batch + 1
 * doubles): [0, batch) norm h^3 sum |psi_j|^2; [batch, 2 batch) Lyapunov
 * functional h^3 (psi_j^* psi_j + f_j^* Q f_j) (Sec. 3, zeroth- and
 * first-order stability proofs; Q = (H_{Gamma,II} H_{II,Gamma})^{-1};
 * equal to the norm for the other orders, the second included, for which
 * the paper states no such functional);
 * [2 batch, 3 batch) h^3 Re <psi_j, H_{I,I} psi_j>; [3 batch] mean-field
 * interaction energy h^3 sum (t0 rho^2/2 + t3 rho^3/3) (0 without it; the
 * Yukawa and Coulomb terms of ABC_MF_SKYRME are not included).
 * Deterministic (fixed-order two-pass reduction). */
abc_status abc_diagnostics(abc_ctx* ctx, const void* psi, const void* aux,
                           const void* V, double* out, void* stream);

/* abc_diagnostics without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, output and kernels as
 * abc_diagnostics; the reduction partials live in a fixed array of the
 * library, one copy per GPU, held until the process ends:
 *   at most 64 orbitals (batch), 64 * 320 * 4 doubles = 640 KiB.
 * A larger batch returns ABC_EINVAL before any work is queued.  The call
 * queues its kernels on the stream and returns without synchronising; it
 * calls no hipMalloc, hipFree or other allocating routine.  Every call on a
 * GPU, from any context, shares that GPU's array: calls that overlap in time
 * on one GPU (other streams, other threads) race and give wrong results;
 * serialise them on one stream.  The array keeps the last call's partials;
 * each call writes every partial it reads first, so nothing has to be
 * cleared. */
abc_status abc_diagnostics_noalloc(abc_ctx* ctx, const void* psi, const void* aux,
                                   const void* V, double* out, void* stream);

/* Number of complex128 elements of the auxiliary buffer (0 unless first or
 * second order; second order: 2 n_Gamma batch). */
size_t abc_aux_elems(const abc_ctx* ctx);

/* Copy a setup product to host memory (for inspection and tests).
 * which = 0: face kernel, R*R*(2w+1)^2 complex128 as [l][l'][p1+w][p2+w];
 * which = 1: box-form matrix, row-major: M (zeroth, n x n), [B | A] (first,
 *            n x 2n) or [[0, I, A1], [B0, B1, B1 A1 + A0]] (second,
 *            2n x 3n, acting on [f; g; E psi]), n = n_Gamma.
 * which = 2: face-form normal-line blocks, a (R*R) then q (R*R) complex128.
 * which = 3: box-form sizes, two complex128: (n_Gamma, r), r the dimension
 *            the second order interpolates in (n_Gamma for the other
 *            orders), then (spectral bound of the boundary block, 0).
 * n = capacity in complex128 elements; returns EINVAL if too small. */
abc_status abc_export(const abc_ctx* ctx, int which, void* host_out, size_t n);

/* Execution path chosen at setup: ABC_PATH_STAGED, ABC_PATH_FUSED (two
 * launches of two stages per step) or ABC_PATH_ONEPASS (one launch per
 * step). */
int abc_path(const abc_ctx* ctx);

/* Bytes of device memory held by the context. */
size_t abc_device_bytes(const abc_ctx* ctx);

/* Message of the last failed call on this thread ("" if none). */
const char* abc_last_error(void);

/* Checkpoint and resume.  abc_state_save writes the state (psi, and aux
 * unless the context has none) of ctx's box to the file `path`: a 128-byte
 * header (magic "ABCSTATE", format version, nx, ny, nz, radius, order, form,
 * dtype, batch, window, fejer, h, dt, s0, s1, s2, the caller's step
 * counter, the byte counts of psi and aux, in native byte order), then psi
 * and aux as stored on the device.  psi and
 * aux are device buffers; the call waits for the stream, copies through host
 * memory and allocates a host buffer of their size.  abc_state_load reads
 * such a file into psi and aux for a context with the same box and
 * parameters (ABC_EINVAL otherwise, naming the first mismatch) and returns
 * the stored step counter in *step (may be NULL).  ABC_EIO if the file cannot
 * be opened, read or written. */
abc_status abc_state_save(abc_ctx* ctx, const void* psi, const void* aux, long long step, const char* path,
                          void* stream);
abc_status abc_state_load(abc_ctx* ctx, void* psi, void* aux, long long* step, const char* path, void* stream);

/* Release everything the context owns (NULL is ignored). */
void abc_destroy(abc_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* ABC_DTN_H */
