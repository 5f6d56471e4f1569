// H2 objective of the first-order interpolation point (Sec. 5: choose s1 as
// the minimiser of ||K(s) - R11(s)||_H2), evaluated for the face form per
// half-space and per transverse Fourier mode theta = (theta1, theta2):
//
//   J(s1) = P^-2 sum_theta (1/2pi) int |k^(theta; i w) - a / (i w - b_w(theta))|^2 dw
//
// k^ is the half-line DtN symbol on the imaginary axis (the limit from
// Re s > 0; R = 1 closed form), a = -i H_gs H_gs^T, and b_w the symbol of the
// windowed kernel of B actually applied at s1 (Theorem 3.2 per mode, built by
// the host face setup).  Modes: the P x P grid 2 pi j / P.  Frequencies:
// w = W0 (tan(phi) - 1), W0 = 3/h^2, phi on N midpoints of (-pi/2, pi/2), with
// weight W0 sec^2(phi) pi / N.  One workgroup per mode sums its frequency
// integral; a single workgroup adds the modes in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "abc_internal.h"

namespace {

constexpr int kT = 256;

// b_w(theta_i, theta_j) = sum_{p, q} k(p, q) exp(-i (p theta_i + q theta_j))
__global__ void __launch_bounds__(kT) h2_symbol_kernel(const double2* __restrict__ ker, int w, int P,
                                                       double2* __restrict__ bw) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P * P) return;
  const int i = e / P, j = e % P;
  const double t1 = 2.0 * M_PI * i / P, t2 = 2.0 * M_PI * j / P;
  const int K = 2 * w + 1;
  double sr = 0, si = 0;
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b) {
      double sn, cs;
      sincos(-((a - w) * t1 + (b - w) * t2), &sn, &cs);
      const double2 k = ker[a * K + b];
      sr += k.x * cs - k.y * sn;
      si += k.x * sn + k.y * cs;
    }
  bw[e] = make_double2(sr, si);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

__global__ void __launch_bounds__(kT) h2_mode_kernel(const double2* __restrict__ bw, int P, int N, double h,
                                                     double2 a, double* __restrict__ part) {
  __shared__ double sh[kT];
  const int e = blockIdx.x;
  const int i = e / P, j = e % P;
  const double h2 = h * h;
  const double tau = ((1.0 - cos(2.0 * M_PI * i / P)) + (1.0 - cos(2.0 * M_PI * j / P))) / h2;
  const double2 b = bw[e];
  const double w0 = 3.0 / h2;
  double acc = 0;
  for (int m = threadIdx.x; m < N; m += blockDim.x) {
    const double phi = -0.5 * M_PI + (m + 0.5) * M_PI / N;
    double sn, cs;
    sincos(phi, &sn, &cs);
    const double om = -w0 + w0 * (sn / cs);
    const double wt = w0 / (cs * cs) * (M_PI / N);
    // decaying root of u^2 - 2 beta u + 1 = 0, beta = 1 + h^2 (tau + om)
    const double beta = 1.0 + h2 * (tau + om);
    double ur, ui = 0;
    if (beta > 1.0) {
      ur = 1.0 / (beta + sqrt(beta * beta - 1.0));
    } else if (beta < -1.0) {
      ur = 1.0 / (beta - sqrt(beta * beta - 1.0));
    } else {
      ur = beta;
      ui = sqrt(1.0 - beta * beta);
    }
    const double kr = -ur / (2.0 * h2), ki = -ui / (2.0 * h2);
    // r = a / (i om - b)
    const double dr = -b.x, di = om - b.y;
    const double inv = 1.0 / (dr * dr + di * di);
    const double rr = (a.x * dr + a.y * di) * inv, ri = (a.y * dr - a.x * di) * inv;
    const double xr = kr - rr, xi = ki - ri;
    acc += wt * (xr * xr + xi * xi);
  }
  const double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) part[e] = tot;
}

__global__ void __launch_bounds__(kT) h2_finish_kernel(const double* __restrict__ part, int count, double scale,
                                                       double* __restrict__ out) {
  __shared__ double sh[kT];
  double acc = 0;
  for (int e = threadIdx.x; e < count; e += blockDim.x) acc += part[e];
  const double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = tot * scale;
}

}  // namespace

abc_status run_h2_objective(const abc_params& p0, const double* s1, int count, int modes, int nodes, double* out,
                            hipStream_t st, std::string& err) {
  const int P = modes;
  std::vector<void*> bufs;
  auto cleanup = [&]() {
    for (void* q : bufs) (void)hipFree(q);
  };
  auto dalloc = [&](void** q, size_t bytes) {
    if (hipMalloc(q, bytes) != hipSuccess) return false;
    bufs.push_back(*q);
    return true;
  };
  const int K = 2 * p0.window + 1;
  void *ker = nullptr, *bw = nullptr, *part = nullptr, *res = nullptr;
  if (!dalloc(&ker, (size_t)K * K * sizeof(double2)) || !dalloc(&bw, (size_t)P * P * sizeof(double2)) ||
      !dalloc(&part, (size_t)P * P * sizeof(double)) || !dalloc(&res, (size_t)count * sizeof(double))) {
    cleanup();
    err = "device allocation for the H2 objective failed";
    return ABC_ENOMEM;
  }
  std::vector<double2> hk((size_t)K * K);
  for (int c = 0; c < count; ++c) {
    abc_params p = p0;
    p.s1 = s1[c];
    abc::FaceOps ops;
    abc_status s = abc::build_face_ops(p, ops, err);
    if (s != ABC_OK) {
      cleanup();
      err = "H2 objective, s1 = " + std::to_string(s1[c]) + ": " + err;
      return s;
    }
    for (size_t q = 0; q < hk.size(); ++q) hk[q] = make_double2(ops.kernel[q].real(), ops.kernel[q].imag());
    // the host copy is reused by the next candidate: wait for this upload
    if (hipMemcpyAsync(ker, hk.data(), hk.size() * sizeof(double2), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      cleanup();
      err = "hipMemcpy failed";
      return ABC_EDEVICE;
    }
    h2_symbol_kernel<<<(P * P + kT - 1) / kT, kT, 0, st>>>(static_cast<const double2*>(ker), p.window, P,
                                                           static_cast<double2*>(bw));
    const double2 a = make_double2(ops.a[0].real(), ops.a[0].imag());
    h2_mode_kernel<<<P * P, kT, 0, st>>>(static_cast<const double2*>(bw), P, nodes, p.h, a,
                                          static_cast<double*>(part));
    h2_finish_kernel<<<1, kT, 0, st>>>(static_cast<const double*>(part), P * P, 1.0 / (2.0 * M_PI * P * P),
                                        static_cast<double*>(res) + c);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(out, res, (size_t)count * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  cleanup();
  if (e != hipSuccess) {
    err = std::string("H2 objective: ") + hipGetErrorString(e);
    return ABC_EDEVICE;
  }
  return ABC_OK;
}
