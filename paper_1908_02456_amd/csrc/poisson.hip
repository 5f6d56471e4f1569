// Long-range TDHF potentials (Sec. 4.3): the Yukawa and Coulomb fields of the
// density rho = sum_j |phi_j|^2 from the Helmholtz and Poisson problems
//
//   (-Delta_h + 1/a^2) W_Y = 4 pi V0 a rho,      -Delta_h W_C = 2 pi e^2 rho,
//
// on the box with the wavefunctions' Laplacian of half-width R and zero
// values outside, solved every step by preconditioned conjugate gradients
// (the paper's method for these problems), FP64 throughout.
//
// Preconditioner: the R = 1 operator -Delta_h + mu^2 with zero values outside
// is diagonalised by the sine transform (DST-I) along each axis, so its
// inverse is three dense n x n transforms, a division by its eigenvalues
// sum_a (2 - 2 cos(pi k_a / (n_a + 1))) / h^2 + mu^2, and three transforms
// back.  Each transform along one axis is a GEMM over all lines (FP64 matrix
// cores through rocBLAS).  It is the exact inverse for R = 1, where CG stops
// after one iteration, and spectrally equivalent to the R = 2, 3 operators.
//
// CG kernels run over a fixed grid of workgroups; every workgroup reduces
// the block partials in the same fixed order (alpha and beta are identical
// everywhere), and the convergence flag is read once per workgroup.  Solves
// start from the previous step's potential unless that start is worse than
// zero.  Either the host reads the flag after each iteration and stops at
// convergence, or (fixed mode) every solve issues a fixed number of
// iterations whose kernels return at once after convergence, with no host
// read, so that a step can be captured in a graph.  Each solve's iteration
// count and whether it converged are added up on the device.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>

#include "abc_internal.h"

namespace {

constexpr int kT = 256;

// scalar slots of PotentialSolver::scal
enum { kRZ0 = 0, kRZ1 = 1, kBB = 2, kDone = 3, kIter = 4, kReset = 5, kRR = 6 };

struct Op {
  int nx, ny, nz;
  long long n;
  double diag;                 // -3 c0 / h^2 + mu^2
  double off[abc::kMaxR + 1];  // -c_k / h^2
};

template <int R>
__device__ __forceinline__ double apply_op(const Op& op, const double* __restrict__ x, long long e) {
  const int ix = (int)(e % op.nx);
  const int iy = (int)((e / op.nx) % op.ny);
  const int iz = (int)(e / ((long long)op.nx * op.ny));
  const long long sy = op.nx, sz = (long long)op.nx * op.ny;
  double acc = op.diag * x[e];
#pragma unroll
  for (int k = 1; k <= R; ++k) {
    double s = 0;
    if (ix + k < op.nx) s += x[e + k];
    if (ix - k >= 0) s += x[e - k];
    if (iy + k < op.ny) s += x[e + k * sy];
    if (iy - k >= 0) s += x[e - k * sy];
    if (iz + k < op.nz) s += x[e + k * sz];
    if (iz - k >= 0) s += x[e - k * sz];
    acc += op.off[k] * s;
  }
  return acc;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// the convergence flag, read once per workgroup (another workgroup of the
// direction update may set it while this one starts)
__device__ __forceinline__ bool block_done(const double* __restrict__ scal) {
  __shared__ int flag;
  if (threadIdx.x == 0) flag = scal[kDone] != 0.0 ? 1 : 0;
  __syncthreads();
  return flag != 0;
}

// sum of nblk partials in a fixed order (every workgroup gets the same value)
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int nblk, double* sh) {
  double a = 0;
  for (int i = threadIdx.x; i < nblk; i += kT) a += part[i];
  return block_sum(a, sh);
}

// b = scale rho; r = b - A x; partials of r.r and b.b
template <int R>
__global__ void __launch_bounds__(kT) cg_init_kernel(Op op, const double* __restrict__ rho, double scale,
                                                     const double* __restrict__ x, double* __restrict__ r,
                                                     double* __restrict__ part, int nblk) {
  __shared__ double sh[kT];
  double rr = 0, bb = 0;
  for (long long e = (long long)blockIdx.x * kT + threadIdx.x; e < op.n; e += (long long)gridDim.x * kT) {
    const double b = scale * rho[e];
    const double re = b - apply_op<R>(op, x, e);
    r[e] = re;
    rr += re * re;
    bb += b * b;
  }
  rr = block_sum(rr, sh);
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rr;
    part[nblk + blockIdx.x] = bb;
  }
}

// one workgroup: the start residual; a start worse than zero is replaced by
// zero (r = b, r.r = b.b); convergence test r.r <= tol^2 b.b
__global__ void __launch_bounds__(kT) cg_start_kernel(const double* __restrict__ part, int nblk, double tol2,
                                                      double* __restrict__ scal) {
  __shared__ double sh[kT];
  const double rr = sum_partials(part, nblk, sh);
  const double bb = sum_partials(part + nblk, nblk, sh);
  if (threadIdx.x == 0) {
    const bool reset = rr > bb;
    const double r0 = reset ? bb : rr;
    scal[kRR] = r0;
    scal[kBB] = bb;
    scal[kReset] = reset ? 1.0 : 0.0;
    scal[kDone] = r0 <= tol2 * bb ? 1.0 : 0.0;
    scal[kIter] = 0.0;
  }
}

// zero start: x = 0, r = b
__global__ void __launch_bounds__(kT) cg_reset_kernel(long long n, const double* __restrict__ rho, double scale,
                                                      double* __restrict__ x, double* __restrict__ r,
                                                      const double* __restrict__ scal) {
  if (scal[kReset] == 0.0) return;
  for (long long e = (long long)blockIdx.x * kT + threadIdx.x; e < n; e += (long long)gridDim.x * kT) {
    x[e] = 0.0;
    r[e] = scale * rho[e];
  }
}

// partials of r.z
__global__ void __launch_bounds__(kT) cg_dot_kernel(long long n, const double* __restrict__ r,
                                                    const double* __restrict__ z, double* __restrict__ part,
                                                    const double* __restrict__ scal) {
  __shared__ double sh[kT];
  if (block_done(scal)) return;
  double rz = 0;
  for (long long e = (long long)blockIdx.x * kT + threadIdx.x; e < n; e += (long long)gridDim.x * kT) rz += r[e] * z[e];
  rz = block_sum(rz, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = rz;
}

// first direction p = z, with r.z
__global__ void __launch_bounds__(kT) cg_first_kernel(long long n, double* __restrict__ p, const double* __restrict__ z,
                                                      const double* __restrict__ part_rz, int nblk,
                                                      double* __restrict__ scal) {
  __shared__ double sh[kT];
  if (block_done(scal)) return;
  const double rz = sum_partials(part_rz, nblk, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) scal[kRZ0] = rz;
  for (long long e = (long long)blockIdx.x * kT + threadIdx.x; e < n; e += (long long)gridDim.x * kT) p[e] = z[e];
}

// q = A p; partials of p.q
template <int R>
__global__ void __launch_bounds__(kT) cg_ap_kernel(Op op, const double* __restrict__ p, double* __restrict__ q,
                                                   double* __restrict__ part, const double* __restrict__ scal) {
  __shared__ double sh[kT];
  if (block_done(scal)) return;
  double pq = 0;
  for (long long e = (long long)blockIdx.x * kT + threadIdx.x; e < op.n; e += (long long)gridDim.x * kT) {
    const double v = apply_op<R>(op, p, e);
    q[e] = v;
    pq += p[e] * v;
  }
  pq = block_sum(pq, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = pq;
}

// alpha = (r.z) / (p.q); x += alpha p; r -= alpha q; partials of r.r
__global__ void __launch_bounds__(kT) cg_x_kernel(long long n, double* __restrict__ x, double* __restrict__ r,
                                                  const double* __restrict__ p, const double* __restrict__ q,
                                                  const double* __restrict__ part_pq, double* __restrict__ part_rr,
                                                  int nblk, const double* __restrict__ scal, int cur) {
  __shared__ double sh[kT];
  if (block_done(scal)) return;
  const double pq = sum_partials(part_pq, nblk, sh);
  const double alpha = scal[kRZ0 + cur] / pq;
  double rr = 0;
  for (long long e = (long long)blockIdx.x * kT + threadIdx.x; e < n; e += (long long)gridDim.x * kT) {
    x[e] += alpha * p[e];
    const double re = r[e] - alpha * q[e];
    r[e] = re;
    rr += re * re;
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = rr;
}

// convergence on r.r; beta = (r'.z') / (r.z); p = z + beta p
__global__ void __launch_bounds__(kT) cg_p_kernel(long long n, double tol2, double* __restrict__ p,
                                                  const double* __restrict__ z, const double* __restrict__ part_rr,
                                                  const double* __restrict__ part_rz, int nblk,
                                                  double* __restrict__ scal, int cur) {
  __shared__ double sh[kT];
  if (block_done(scal)) return;
  const double rrn = sum_partials(part_rr, nblk, sh);
  const double rzn = sum_partials(part_rz, nblk, sh);
  const bool done = rrn <= tol2 * scal[kBB];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[kRR] = rrn;
    scal[kRZ0 + 1 - cur] = rzn;
    scal[kIter] += 1.0;
    if (done) scal[kDone] = 1.0;
  }
  if (done) return;
  const double beta = rzn / scal[kRZ0 + cur];
  for (long long e = (long long)blockIdx.x * kT + threadIdx.x; e < n; e += (long long)gridDim.x * kT)
    p[e] = z[e] + beta * p[e];
}

// end of a solve: its iterations into tally[field], an unconverged solve
// into tally[2]
__global__ void cg_tally_kernel(const double* __restrict__ scal, double* __restrict__ tally, int field) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    tally[field] += scal[kIter];
    if (scal[kDone] == 0.0) tally[2] += 1.0;
  }
}

// divide the sine coefficients by the eigenvalues of the R = 1 operator
// (-Delta_h + mu^2, zero outside) times the transforms' normalisation
__global__ void __launch_bounds__(kT) dst_scale_kernel(double* __restrict__ a, const double* __restrict__ ex,
                                                       const double* __restrict__ ey, const double* __restrict__ ez,
                                                       int nx, int ny, int nz, double mu2, double norm) {
  const long long e = (long long)blockIdx.x * kT + threadIdx.x;
  if (e >= (long long)nx * ny * nz) return;
  const int ix = (int)(e % nx), iy = (int)((e / nx) % ny), iz = (int)(e / ((long long)nx * ny));
  a[e] *= norm / (ex[ix] + ey[iy] + ez[iz] + mu2);
}

// One sine transform of [z][y][x] data along all three axes: three FP64
// GEMMs with the symmetric DST-I matrices (x: S_x X; y: per z-plane X S_y;
// z: X S_z in the column-major views), in -> out through tmp.
rocblas_status dst3(const PotentialSolver& ps, const double* in, double* tmp, double* out) {
  rocblas_handle hb = static_cast<rocblas_handle>(ps.blas);
  const int nx = ps.nx, ny = ps.ny, nz = ps.nz;
  const double one = 1.0, zero = 0.0;
  rocblas_status rs = rocblas_dgemm(hb, rocblas_operation_none, rocblas_operation_none, nx, ny * nz, nx, &one, ps.sx,
                                    nx, in, nx, &zero, out, nx);
  if (rs == rocblas_status_success)
    rs = rocblas_dgemm_strided_batched(hb, rocblas_operation_none, rocblas_operation_none, nx, ny, ny, &one, out, nx,
                                       (rocblas_stride)nx * ny, ps.sy, ny, 0, &zero, tmp, nx, (rocblas_stride)nx * ny,
                                       nz);
  if (rs == rocblas_status_success)
    rs = rocblas_dgemm(hb, rocblas_operation_none, rocblas_operation_none, nx * ny, nz, nz, &one, tmp, nx * ny, ps.sz,
                       nz, &zero, out, nx * ny);
  return rs;
}

// z = M^{-1} r with M the R = 1 operator: exact for R = 1, spectrally
// equivalent for R = 2, 3
hipError_t dst_precond(const PotentialSolver& ps, double mu2, const double* r, double* z, hipStream_t st) {
  if (rocblas_set_stream(static_cast<rocblas_handle>(ps.blas), st) != rocblas_status_success) return hipErrorUnknown;
  if (dst3(ps, r, ps.t1, ps.t2) != rocblas_status_success) return hipErrorLaunchFailure;
  const long long n = (long long)ps.nx * ps.ny * ps.nz;
  const double norm = (2.0 / (ps.nx + 1)) * (2.0 / (ps.ny + 1)) * (2.0 / (ps.nz + 1));
  dst_scale_kernel<<<(unsigned)((n + kT - 1) / kT), kT, 0, st>>>(ps.t2, ps.ex, ps.ey, ps.ez, ps.nx, ps.ny, ps.nz,
                                                                  mu2, norm);
  if (dst3(ps, ps.t2, ps.t1, z) != rocblas_status_success) return hipErrorLaunchFailure;
  return hipGetLastError();
}

template <int R>
hipError_t cg_solve(const Op& op, double mu2, const double* rho, double scale, double* x, PotentialSolver& ps,
                    hipStream_t st, long long* iters, int field) {
  const int nb = ps.nblk;
  double* part_a = ps.part;
  double* part_b = ps.part + nb;
  double* part_c = ps.part + 2 * nb;
  const double tol2 = ps.tol * ps.tol;
  cg_init_kernel<R><<<nb, kT, 0, st>>>(op, rho, scale, x, ps.r, part_a, nb);
  cg_start_kernel<<<1, kT, 0, st>>>(part_a, nb, tol2, ps.scal);
  cg_reset_kernel<<<nb, kT, 0, st>>>(op.n, rho, scale, x, ps.r, ps.scal);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = dst_precond(ps, mu2, ps.r, ps.z, st);
  if (e == hipSuccess) {
    cg_dot_kernel<<<nb, kT, 0, st>>>(op.n, ps.r, ps.z, part_c, ps.scal);
    cg_first_kernel<<<nb, kT, 0, st>>>(op.n, ps.p, ps.z, part_c, nb, ps.scal);
    e = hipGetLastError();
  }
  if (ps.fixed > 0) {
    // a fixed number of iterations, no host read; after convergence every
    // CG kernel returns at once (the preconditioner's transforms still run)
    for (int it = 0; e == hipSuccess && it < ps.fixed; ++it) {
      const int cur = it & 1;
      cg_ap_kernel<R><<<nb, kT, 0, st>>>(op, ps.p, ps.q, part_a, ps.scal);
      cg_x_kernel<<<nb, kT, 0, st>>>(op.n, x, ps.r, ps.p, ps.q, part_a, part_b, nb, ps.scal, cur);
      e = hipGetLastError();
      if (e == hipSuccess) e = dst_precond(ps, mu2, ps.r, ps.z, st);
      if (e == hipSuccess) {
        cg_dot_kernel<<<nb, kT, 0, st>>>(op.n, ps.r, ps.z, part_c, ps.scal);
        cg_p_kernel<<<nb, kT, 0, st>>>(op.n, tol2, ps.p, ps.z, part_b, part_c, nb, ps.scal, cur);
        e = hipGetLastError();
      }
    }
    if (e == hipSuccess) {
      cg_tally_kernel<<<1, 64, 0, st>>>(ps.scal, ps.tally, field);
      e = hipGetLastError();
    }
    return e;
  }
  if (e == hipSuccess) e = hipMemcpyAsync(ps.host, ps.scal + kDone, 2 * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  for (int it = 0; e == hipSuccess && ps.host[0] == 0.0 && it < ps.maxit; ++it) {
    const int cur = it & 1;
    cg_ap_kernel<R><<<nb, kT, 0, st>>>(op, ps.p, ps.q, part_a, ps.scal);
    cg_x_kernel<<<nb, kT, 0, st>>>(op.n, x, ps.r, ps.p, ps.q, part_a, part_b, nb, ps.scal, cur);
    e = hipGetLastError();
    if (e == hipSuccess) e = dst_precond(ps, mu2, ps.r, ps.z, st);
    if (e == hipSuccess) {
      cg_dot_kernel<<<nb, kT, 0, st>>>(op.n, ps.r, ps.z, part_c, ps.scal);
      cg_p_kernel<<<nb, kT, 0, st>>>(op.n, tol2, ps.p, ps.z, part_b, part_c, nb, ps.scal, cur);
      e = hipGetLastError();
    }
    // few iterations with this preconditioner: read the flag after each
    if (e == hipSuccess) e = hipMemcpyAsync(ps.host, ps.scal + kDone, 2 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  if (e == hipSuccess) *iters += (long long)ps.host[1];
  if (e == hipSuccess) {
    cg_tally_kernel<<<1, 64, 0, st>>>(ps.scal, ps.tally, field);
    e = hipGetLastError();
  }
  return e;
}

Op make_op(const PotentialSolver& ps, double mu2) {
  Op op{};
  op.nx = ps.nx;
  op.ny = ps.ny;
  op.nz = ps.nz;
  op.n = (long long)ps.nx * ps.ny * ps.nz;
  const double ih2 = 1.0 / (ps.h * ps.h);
  op.diag = -3.0 * ps.c[0] * ih2 + mu2;
  for (int k = 1; k <= ps.R; ++k) op.off[k] = -ps.c[k] * ih2;
  return op;
}

template <typename C>
__global__ void __launch_bounds__(kT) rho_kernel(const C* __restrict__ psi, long long n, int B, int soa,
                                                 double* __restrict__ rho) {
  const long long p = (long long)blockIdx.x * kT + threadIdx.x;
  if (p >= n) return;
  double s = 0;
  for (int b = 0; b < B; ++b) {
    const C v = soa ? psi[(long long)b * n + p] : psi[p * B + b];
    s += (double)v.x * v.x + (double)v.y * v.y;
  }
  rho[p] = s;
}

template <typename T>
__global__ void __launch_bounds__(kT) veff_kernel(const T* __restrict__ V, const double* __restrict__ rho,
                                                  const double* __restrict__ wy, const double* __restrict__ wc,
                                                  long long n, double t0, double t3, T* __restrict__ veff) {
  const long long p = (long long)blockIdx.x * kT + threadIdx.x;
  if (p >= n) return;
  const double r = rho[p];
  double u = t0 * r + t3 * r * r;
  if (wy) u += wy[p];
  if (wc) u += wc[p];
  veff[p] = (T)((V ? (double)V[p] : 0.0) + u);
}

template <int R>
hipError_t solve_both(PotentialSolver& ps, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (ps.v0 != 0.0) {
    const Op op = make_op(ps, 1.0 / (ps.a * ps.a));
    e = cg_solve<R>(op, 1.0 / (ps.a * ps.a), ps.rho, 4.0 * M_PI * ps.v0 * ps.a, ps.wy, ps, st, &ps.iters_y, 0);
  }
  if (e == hipSuccess && ps.e2 != 0.0) {
    const Op op = make_op(ps, 0.0);
    e = cg_solve<R>(op, 0.0, ps.rho, 2.0 * M_PI * ps.e2, ps.wc, ps, st, &ps.iters_c, 1);
  }
  if (e == hipSuccess) ++ps.solves;
  return e;
}

}  // namespace

// one preconditioner application on zero data at setup, so that rocBLAS
// finishes its lazy initialisation before the first step
hipError_t potential_warmup(PotentialSolver& ps) {
  const size_t n = (size_t)ps.nx * ps.ny * ps.nz;
  hipError_t e = hipMemset(ps.r, 0, n * sizeof(double));
  if (e == hipSuccess) e = dst_precond(ps, 0.0, ps.r, ps.z, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return e;
}

// V + t0 rho + t3 rho^2 + W_Y + W_C for the state psi (AoS [point][orbital]
// or SoA [orbital][point] orbital arrays), into veff of the state's real type
hipError_t skyrme_veff(PotentialSolver& ps, const void* psi, bool soa, int B, bool c64, const void* V, void* veff,
                       double t0, double t3, hipStream_t st, abc_timer* tm) {
  const long long n = (long long)ps.nx * ps.ny * ps.nz;
  const unsigned blocks = (unsigned)((n + kT - 1) / kT);
  if (c64)
    rho_kernel<float2><<<blocks, kT, 0, st>>>(static_cast<const float2*>(psi), n, B, soa ? 1 : 0, ps.rho);
  else
    rho_kernel<double2><<<blocks, kT, 0, st>>>(static_cast<const double2*>(psi), n, B, soa ? 1 : 0, ps.rho);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (ps.R) {
    case 1: e = solve_both<1>(ps, st); break;
    case 2: e = solve_both<2>(ps, st); break;
    case 3: e = solve_both<3>(ps, st); break;
    default: e = hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  const double* wy = ps.v0 != 0.0 ? ps.wy : nullptr;
  const double* wc = ps.e2 != 0.0 ? ps.wc : nullptr;
  if (c64)
    abc_launch_kernel(tm, "meanfield", veff_kernel<float>, dim3(blocks), dim3(kT), st, static_cast<const float*>(V),
                      (const double*)ps.rho, wy, wc, n, t0, t3, static_cast<float*>(veff));
  else
    abc_launch_kernel(tm, "meanfield", veff_kernel<double>, dim3(blocks), dim3(kT), st,
                      static_cast<const double*>(V), (const double*)ps.rho, wy, wc, n, t0, t3,
                      static_cast<double*>(veff));
  return hipGetLastError();
}
