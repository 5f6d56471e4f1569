// Long-range TDHF potentials (Sec. 4.3): the Yukawa and Coulomb fields of the
// density rho = sum_j |phi_j|^2 from the Helmholtz and Poisson problems
//
//   (-Delta_h + 1/a^2) W_Y = 4 pi V0 a rho,      -Delta_h W_C = 2 pi e^2 rho,
//
// on the box with the wavefunctions' Laplacian of half-width R and zero
// values outside, solved every step by preconditioned conjugate gradients
// (the paper's method for these problems; the Jacobi preconditioner of this
// constant-coefficient operator is a constant scaling).  FP64 throughout.
// Each iteration is three launches over a fixed grid of workgroups: q = A p
// with partial sums of p.q; the x, r update (every workgroup reduces the
// partials in the same fixed order, so alpha is identical everywhere) with
// partial sums of r.r; and the direction update, which also decides
// convergence.  Solves start from the previous step's potential unless that
// start is worse than zero.  The host reads the convergence flag every
// kChunk iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "abc_internal.h"

namespace {

constexpr int kT = 256;
constexpr int kChunk = 8;

// scalar slots of PotentialSolver::scal
enum { kRR0 = 0, kRR1 = 1, kBB = 2, kDone = 3, kIter = 4, kReset = 5 };

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

// b = scale rho; r = b - A x; p = r / d; partials of r.r and b.b
template <int R>
__global__ void __launch_bounds__(kT) cg_init_kernel(Op op, const double* __restrict__ rho, double scale,
                                                     const double* __restrict__ x, double* __restrict__ r,
                                                     double* __restrict__ p, double* __restrict__ part, int nblk) {
  __shared__ double sh[kT];
  double rr = 0, bb = 0;
  const double dinv = 1.0 / op.diag;
  for (long long e = (long long)blockIdx.x * kT + threadIdx.x; e < op.n; e += (long long)gridDim.x * kT) {
    const double b = scale * rho[e];
    const double re = b - apply_op<R>(op, x, e);
    r[e] = re;
    p[e] = re * dinv;
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
// zero (r = b, rr = bb); convergence test rr <= tol^2 bb
__global__ void __launch_bounds__(kT) cg_start_kernel(const double* __restrict__ part, int nblk, double tol2,
                                                      double* __restrict__ scal) {
  __shared__ double sh[kT];
  const double rr = sum_partials(part, nblk, sh);
  const double bb = sum_partials(part + nblk, nblk, sh);
  if (threadIdx.x == 0) {
    const bool reset = rr > bb;
    const double r0 = reset ? bb : rr;
    scal[kRR0] = r0;
    scal[kBB] = bb;
    scal[kReset] = reset ? 1.0 : 0.0;
    scal[kDone] = r0 <= tol2 * bb ? 1.0 : 0.0;
    scal[kIter] = 0.0;
  }
}

// zero start: x = 0, r = b, p = b / d
__global__ void __launch_bounds__(kT) cg_reset_kernel(Op op, const double* __restrict__ rho, double scale,
                                                      double* __restrict__ x, double* __restrict__ r,
                                                      double* __restrict__ p, const double* __restrict__ scal) {
  if (scal[kReset] == 0.0) return;
  const double dinv = 1.0 / op.diag;
  for (long long e = (long long)blockIdx.x * kT + threadIdx.x; e < op.n; e += (long long)gridDim.x * kT) {
    const double b = scale * rho[e];
    x[e] = 0.0;
    r[e] = b;
    p[e] = b * dinv;
  }
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

// alpha = (r.z) / (p.q) with z = r / d; x += alpha p; r -= alpha q; partials of r.r
__global__ void __launch_bounds__(kT) cg_x_kernel(long long n, double dinv, double* __restrict__ x,
                                                  double* __restrict__ r, const double* __restrict__ p,
                                                  const double* __restrict__ q, const double* __restrict__ part_pq,
                                                  double* __restrict__ part_rr, int nblk,
                                                  const double* __restrict__ scal, int cur) {
  __shared__ double sh[kT];
  if (block_done(scal)) return;
  const double pq = sum_partials(part_pq, nblk, sh);
  const double alpha = scal[kRR0 + cur] * dinv / pq;
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

// beta = (r'.z') / (r.z); p = r / d + beta p, unless converged
__global__ void __launch_bounds__(kT) cg_p_kernel(long long n, double dinv, double tol2, double* __restrict__ p,
                                                  const double* __restrict__ r, const double* __restrict__ part_rr,
                                                  int nblk, double* __restrict__ scal, int cur) {
  __shared__ double sh[kT];
  if (block_done(scal)) return;
  const double rrn = sum_partials(part_rr, nblk, sh);
  const bool done = rrn <= tol2 * scal[kBB];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[kRR0 + 1 - cur] = rrn;
    scal[kIter] += 1.0;
    if (done) scal[kDone] = 1.0;
  }
  if (done) return;
  const double beta = rrn / scal[kRR0 + cur];
  for (long long e = (long long)blockIdx.x * kT + threadIdx.x; e < n; e += (long long)gridDim.x * kT)
    p[e] = r[e] * dinv + beta * p[e];
}

template <int R>
hipError_t cg_solve(const Op& op, const double* rho, double scale, double* x, PotentialSolver& ps, hipStream_t st,
                    long long* iters) {
  const int nb = ps.nblk;
  double* part_a = ps.part;
  double* part_b = ps.part + 2 * nb;
  const double dinv = 1.0 / op.diag, tol2 = ps.tol * ps.tol;
  cg_init_kernel<R><<<nb, kT, 0, st>>>(op, rho, scale, x, ps.r, ps.p, part_a, nb);
  cg_start_kernel<<<1, kT, 0, st>>>(part_a, nb, tol2, ps.scal);
  cg_reset_kernel<<<nb, kT, 0, st>>>(op, rho, scale, x, ps.r, ps.p, ps.scal);
  hipError_t e = hipGetLastError();
  int it = 0;
  while (e == hipSuccess && it < ps.maxit) {
    const int m = std::min(kChunk, ps.maxit - it);
    for (int k = 0; k < m; ++k) {
      const int cur = (it + k) & 1;
      cg_ap_kernel<R><<<nb, kT, 0, st>>>(op, ps.p, ps.q, part_a, ps.scal);
      cg_x_kernel<<<nb, kT, 0, st>>>(op.n, dinv, x, ps.r, ps.p, ps.q, part_a, part_b, nb, ps.scal, cur);
      cg_p_kernel<<<nb, kT, 0, st>>>(op.n, dinv, tol2, ps.p, ps.r, part_b, nb, ps.scal, cur);
    }
    it += m;
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(ps.host, ps.scal + kDone, 2 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && ps.host[0] != 0.0) break;
  }
  if (e == hipSuccess) *iters += (long long)ps.host[1];
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
    e = cg_solve<R>(op, ps.rho, 4.0 * M_PI * ps.v0 * ps.a, ps.wy, ps, st, &ps.iters_y);
  }
  if (e == hipSuccess && ps.e2 != 0.0) {
    const Op op = make_op(ps, 0.0);
    e = cg_solve<R>(op, ps.rho, 2.0 * M_PI * ps.e2, ps.wc, ps, st, &ps.iters_c);
  }
  if (e == hipSuccess) ++ps.solves;
  return e;
}

}  // namespace

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
