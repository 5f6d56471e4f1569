// Discrete adjoint of n Taylor-4 steps (reverse mode), complex128.
//
// The step (Sec. 4) applied to the linear dynamics of Sec. 3 is the matrix
// polynomial P(dt L) = sum_{k<=4} (dt L)^k / k! of the generator L, so for a
// real objective J(psi_N) with gradient convention g = dJ/dRe + i dJ/dIm:
//   lambda_n = P(dt L^H) lambda_{n+1},
// which is one staged step with the adjoint operator set La: time step -dt,
// conjugate-transposed boundary kernels, and for the first-order condition
// (R = 1) the auxiliary variable rescaled by -i conj(a) so that L^H keeps the
// forward structure with a -> -conj(a), B -> -B^H.
//
// Potential gradient: dL = -i dV on the psi block, so with the sum-form stage
// vectors z_m = dt^m/m! L^m z_n (forward, recomputed from checkpoints) and
// y_j = dt^j/j! (L^H)^j lambda_{n+1} (adjoint), the derivative of the
// polynomial gives
//   dJ/dV_p += dt sum_{j+m<=3} j! m! / (j+m+1)! Im(conj(y_j[p]) z_m[p]).
//
// Checkpoints every `stride` steps (default ceil(sqrt(n))), taken during a
// forward sweep on the fastest available path; each segment is recomputed
// once, keeping every step's state and its intermediates (the two-stage fused
// kernels' Horner intermediates where they apply, else the staged kernels'
// stage vectors), then walked backwards with one adjoint step per step.  With
// stride >= n there is one segment, kept whole: its recompute is the forward
// run (4 + 3 psi-sized vectors per step in memory, no separate sweep).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "abc_internal.h"
#include "fused.h"

using abc::Geometry;

namespace {

constexpr int kBlock = 256;

struct Stencil {
  double diag;
  double off[abc::kMaxR + 1];
};

// J contribution, lambda_N and the explicit dJ/dV of the objective at psi_N.
// objective 0: J = h^3 sum |psi|^2, lambda = 2 h^3 psi, dJ/dV = 0;
// objective 1: J = h^3 Re <psi, H psi>, lambda = 2 h^3 H psi, dJ/dV = h^3 |psi|^2.
template <int R, bool PER>
__global__ void __launch_bounds__(kBlock) objective_kernel(const double2* __restrict__ psi,
                                                           const double* __restrict__ V, Geometry g, Stencil sc,
                                                           double h3, int objective, double2* __restrict__ lam,
                                                           double* __restrict__ gV, double* __restrict__ partial) {
  __shared__ double red[kBlock];
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double contrib = 0;
  if (p < g.npts) {
    const int x = (int)(p % g.nx), y = (int)((p / g.nx) % g.ny), z = (int)(p / ((long long)g.nx * g.ny));
    const double2 c = psi[p];
    if (objective == 0) {
      contrib = h3 * (c.x * c.x + c.y * c.y);
      lam[p] = make_double2(2 * h3 * c.x, 2 * h3 * c.y);
      gV[p] = 0;
    } else {
      double hr = sc.diag * c.x, hi = sc.diag * c.y;
      auto at = [&](int xx, int yy, int zz, double w) {
        if (PER) {
          xx = (xx % g.nx + g.nx) % g.nx;
          yy = (yy % g.ny + g.ny) % g.ny;
          zz = (zz % g.nz + g.nz) % g.nz;
        } else if (xx < 0 || xx >= g.nx || yy < 0 || yy >= g.ny || zz < 0 || zz >= g.nz) {
          return;
        }
        const double2 v = psi[((long long)zz * g.ny + yy) * g.nx + xx];
        hr += w * v.x;
        hi += w * v.y;
      };
#pragma unroll
      for (int k = 1; k <= R; ++k) {
        const double w = sc.off[k];
        at(x + k, y, z, w);
        at(x - k, y, z, w);
        at(x, y + k, z, w);
        at(x, y - k, z, w);
        at(x, y, z + k, w);
        at(x, y, z - k, w);
      }
      const double v = V ? V[p] : 0.0;
      hr += v * c.x;
      hi += v * c.y;
      contrib = h3 * (c.x * hr + c.y * hi);
      lam[p] = make_double2(2 * h3 * hr, 2 * h3 * hi);
      gV[p] = h3 * (c.x * c.x + c.y * c.y);
    }
  }
  red[threadIdx.x] = contrib;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// fixed-order sum of the block partials (one workgroup)
__global__ void __launch_bounds__(kBlock) sum_kernel(const double* __restrict__ partial, int n,
                                                     double* __restrict__ out) {
  __shared__ double red[kBlock];
  double s = 0;
  for (int i = threadIdx.x; i < n; i += kBlock) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = kBlock / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// gV += dt sum_{j+m<=3} j! m!/(j+m+1)! Im(conj(y_j) z_m)
__global__ void __launch_bounds__(kBlock) vgrad_kernel(double* __restrict__ gV, const double2* __restrict__ y0,
                                                       const double2* __restrict__ y1, const double2* __restrict__ y2,
                                                       const double2* __restrict__ y3, const double2* __restrict__ z0,
                                                       const double2* __restrict__ z1, const double2* __restrict__ z2,
                                                       const double2* __restrict__ z3, long long n, double dt) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double2 y[4] = {y0[p], y1[p], y2[p], y3[p]};
  const double2 z[4] = {z0[p], z1[p], z2[p], z3[p]};
  // Beta(j+1, m+1) for j + m <= 3
  constexpr double w[4][4] = {{1.0, 1.0 / 2, 1.0 / 3, 1.0 / 4},
                              {1.0 / 2, 1.0 / 6, 1.0 / 12, 0},
                              {1.0 / 3, 1.0 / 12, 0, 0},
                              {1.0 / 4, 0, 0, 0}};
  double acc = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int m = 0; m + j < 4; ++m) acc += w[j][m] * (y[j].x * z[m].y - y[j].y * z[m].x);
  gV[p] += dt * acc;
}

// The same with both steps in Horner form.  Forward: u3 = z + (dt/4) L z,
// u2 = z + (dt/3) L u3, u1 = z + (dt/2) L u2, z' = z + dt L u1; differentiating
// the recursion and moving each L to the adjoint side gives
//   gV += dt Im(conj(y_0) u1) + dt/2 Im(conj(y_1) u2) + dt/3 Im(conj(y_2) u3)
//         + dt/4 Im(conj(y_3) z),
// with y_j the adjoint's sum-form vectors as above (y_0 = lambda).  The
// adjoint step's own Horner intermediates w3 = l + (dt/4) M l, w2 = l +
// (dt/3) M w3, w1 = l + (dt/2) M w2 (M = L^H, l = lambda), kept as the
// increments d_k = w_k - l, give those back:
//   y1 = 4 d3,  y2 = 6 d2 - 8 d3,  y3 = 4 d1 - 8 d2 + 8/3 d3.
__global__ void __launch_bounds__(kBlock) vgrad_horner2_kernel(
    double* __restrict__ gV, const double2* __restrict__ lam, const double2* __restrict__ w1,
    const double2* __restrict__ w2, const double2* __restrict__ w3, const double2* __restrict__ u1,
    const double2* __restrict__ u2, const double2* __restrict__ u3, const double2* __restrict__ z0, long long n,
    double dt) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double2 d1 = w1[p], d2 = w2[p], d3 = w3[p];
  double2 a[4];
  a[0] = lam[p];
  a[1] = make_double2(4.0 * d3.x, 4.0 * d3.y);
  a[2] = make_double2(6.0 * d2.x - 8.0 * d3.x, 6.0 * d2.y - 8.0 * d3.y);
  a[3] = make_double2(4.0 * d1.x - 8.0 * d2.x + (8.0 / 3.0) * d3.x, 4.0 * d1.y - 8.0 * d2.y + (8.0 / 3.0) * d3.y);
  const double2 b[4] = {u1[p], u2[p], u3[p], z0[p]};
  double acc = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) acc += (a[j].x * b[j].y - a[j].y * b[j].x) / (double)(j + 1);
  gV[p] += dt * acc;
}

template <int R, bool PER>
hipError_t launch_objective(const abc_launch& L, const double2* psi, const double* V, int objective, double2* lam,
                            double* gV, double* partial, double* J, hipStream_t st) {
  const Geometry& g = L.g;
  Stencil sc{};
  const double s = 1.0 / (2.0 * L.h * L.h);
  sc.diag = -3.0 * L.c[0] * s;
  for (int k = 1; k <= R; ++k) sc.off[k] = -L.c[k] * s;
  const int nb = (int)((g.npts + kBlock - 1) / kBlock);
  objective_kernel<R, PER><<<nb, kBlock, 0, st>>>(psi, V, g, sc, L.h * L.h * L.h, objective, lam, gV, partial);
  sum_kernel<<<1, kBlock, 0, st>>>(partial, nb, J);
  return hipGetLastError();
}

hipError_t objective(const abc_launch& L, const double2* psi, const double* V, int objective, double2* lam,
                     double* gV, double* partial, double* J, hipStream_t st) {
  const bool per = L.periodic != 0;
  switch (L.g.R) {
    case 1: return per ? launch_objective<1, true>(L, psi, V, objective, lam, gV, partial, J, st)
                       : launch_objective<1, false>(L, psi, V, objective, lam, gV, partial, J, st);
    case 2: return per ? launch_objective<2, true>(L, psi, V, objective, lam, gV, partial, J, st)
                       : launch_objective<2, false>(L, psi, V, objective, lam, gV, partial, J, st);
    case 3: return per ? launch_objective<3, true>(L, psi, V, objective, lam, gV, partial, J, st)
                       : launch_objective<3, false>(L, psi, V, objective, lam, gV, partial, J, st);
  }
  return hipErrorInvalidValue;
}

// one device allocation carved into the adjoint's buffers, freed on exit
struct Arena {
  char* base = nullptr;
  size_t used = 0, cap = 0;
  ~Arena() {
    if (base) hipFree(base);
  }
  template <typename P>
  P* take(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    P* p = reinterpret_cast<P*>(base + used);
    used += bytes;
    return p;
  }
};

}  // namespace

abc_status run_adjoint(const abc_launch& L, const abc_launch& La, const abc_scratch& S, const abc_adjoint_args& a,
                       hipStream_t st, std::string& err) {
  const Geometry& g = L.g;
  const int N = a.n_steps;
  const int stride = a.stride > 0 ? a.stride : std::max(1, (int)std::ceil(std::sqrt((double)std::max(N, 1))));
  const int nck = N > 0 ? (N + stride - 1) / stride : 0;
  const int nseg = N > 0 ? std::min(stride, N) : 0;
  const size_t np = (size_t)g.npts;
  const size_t nf = (L.order == ABC_FIRST) ? (size_t)g.face_off[6] : 0;
  const size_t pb = np * sizeof(double2), fb = std::max<size_t>(nf, 1) * sizeof(double2);
  const size_t round = 256;
  const int nb = (int)((np + kBlock - 1) / kBlock);
  // psi-sized: X, lam, y0, 3 adjoint stage vectors, checkpoints, segment
  // states and 3 forward stage vectors per segment step
  const size_t npsi = 6 + (size_t)nck + nseg + 3 * (size_t)nseg;
  const size_t total = npsi * (pb + round) + (3 + (size_t)nck + nseg) * (fb + round) +
                       ((size_t)nb + 1) * sizeof(double) + 2 * round;
  Arena ar;
  hipError_t e = hipMalloc(&ar.base, total);
  if (e != hipSuccess) {
    err = std::string("adjoint buffers (") + std::to_string(total) + " bytes): " + hipGetErrorString(e);
    return ABC_ENOMEM;
  }
  ar.cap = total;
  double2* X = ar.take<double2>(pb);
  double2* lam = ar.take<double2>(pb);
  double2* y0 = ar.take<double2>(pb);
  void* ky[3];
  for (int i = 0; i < 3; ++i) ky[i] = ar.take<double2>(pb);
  std::vector<double2*> ckp(nck), seg(nseg);
  for (auto& q : ckp) q = ar.take<double2>(pb);
  for (auto& q : seg) q = ar.take<double2>(pb);
  std::vector<void*> kz(3 * (size_t)nseg);
  for (auto& q : kz) q = ar.take<double2>(pb);
  double2* fX = ar.take<double2>(fb);
  double2* mu = ar.take<double2>(fb);
  double2* mu2 = ar.take<double2>(fb);  // the adjoint aux's second buffer (fused adjoint step, out of place)
  std::vector<double2*> ckf(nck), segf(nseg);
  for (auto& q : ckf) q = ar.take<double2>(fb);
  for (auto& q : segf) q = ar.take<double2>(fb);
  double* partial = ar.take<double>((size_t)nb * sizeof(double));
  double* Jd = ar.take<double>(sizeof(double));
  double2* aux = nf ? fX : nullptr;
  const double* V = static_cast<const double*>(a.V);

#define ABC_TRY(x)                                       \
  do {                                                   \
    hipError_t e_ = (x);                                 \
    if (e_ != hipSuccess) {                              \
      err = std::string(#x) + ": " + hipGetErrorString(e_); \
      return ABC_EDEVICE;                                \
    }                                                    \
  } while (0)

  // a step that keeps its intermediates: the two-stage fused kernels (Horner
  // form, u1 u2 u3 kept) wherever they cover the operators, else the staged
  // kernels (sum form, z1 z2 z3 kept); the V gradient is formed to match
  const bool horner = a.use_fused && !L.fused_shell && L.w == 0 && g.R == 1 && !L.periodic;
  auto step_keeping = [&](int i, const double2* yin, const double2* fin, double2* yout, double2* fout) {
    if (horner) return launch_step_fused_keep(L, S, yin, fin, yout, fout, V, &kz[3 * (size_t)i], st);
    return launch_step_staged(L, S, yout, fout, V, 1, st, nullptr, &kz[3 * (size_t)i], yin, fin);
  };

  // forward sweep with checkpoints; with one segment (stride >= n: every
  // state and stage vector kept) the segment's own recompute below is the
  // forward run, and no separate sweep is made
  ABC_TRY(hipMemcpyAsync(X, a.psi0, pb, hipMemcpyDeviceToDevice, st));
  if (nf) ABC_TRY(hipMemsetAsync(fX, 0, nf * sizeof(double2), st));
  const bool single = nck == 1;
  if (single) {
    ABC_TRY(hipMemcpyAsync(ckp[0], X, pb, hipMemcpyDeviceToDevice, st));
    if (nf) ABC_TRY(hipMemcpyAsync(ckf[0], fX, nf * sizeof(double2), hipMemcpyDeviceToDevice, st));
    ABC_TRY(hipMemcpyAsync(seg[0], ckp[0], pb, hipMemcpyDeviceToDevice, st));
    if (nf) ABC_TRY(hipMemcpyAsync(segf[0], ckf[0], nf * sizeof(double2), hipMemcpyDeviceToDevice, st));
    for (int i = 0; i < N; ++i) {
      double2* next = i + 1 < N ? seg[i + 1] : X;
      double2* nextf = i + 1 < N ? segf[i + 1] : fX;
      ABC_TRY(step_keeping(i, seg[i], nf ? segf[i] : nullptr, next, nf ? nextf : nullptr));
    }
  }
  for (int c = 0; c < nck && !single; ++c) {
    ABC_TRY(hipMemcpyAsync(ckp[c], X, pb, hipMemcpyDeviceToDevice, st));
    if (nf) ABC_TRY(hipMemcpyAsync(ckf[c], fX, nf * sizeof(double2), hipMemcpyDeviceToDevice, st));
    const int k = std::min(stride, N - c * stride);
    ABC_TRY(a.use_fused ? launch_step_fused(L, S, X, aux, V, k, st) : launch_step_staged(L, S, X, aux, V, k, st));
  }
  // objective at psi_N; the adjoint aux starts at zero
  ABC_TRY(objective(L, X, V, a.objective, lam, a.grad_V, partial, Jd, st));
  if (nf) ABC_TRY(hipMemsetAsync(mu, 0, nf * sizeof(double2), st));
  const long long npl = (long long)np;
  const unsigned gb = (unsigned)((np + kBlock - 1) / kBlock);
  // backward over segments; lambda alternates between lam and y0, so the
  // value before each adjoint step stays where the V gradient reads it
  double2* lcur = lam;
  double2* lnext = y0;
  for (int c = nck - 1; c >= 0; --c) {
    const int s0 = c * stride, len = std::min(stride, N - s0);
    // recompute the segment, keeping each step's state and stage vectors
    // (already there with one segment)
    if (!single) ABC_TRY(hipMemcpyAsync(seg[0], ckp[c], pb, hipMemcpyDeviceToDevice, st));
    if (nf && !single) ABC_TRY(hipMemcpyAsync(segf[0], ckf[c], nf * sizeof(double2), hipMemcpyDeviceToDevice, st));
    for (int i = 0; i < len && !single; ++i) {
      // one step from seg[i] (and segf[i]) into the next slot, out of place
      double2* next = i + 1 < len ? seg[i + 1] : X;
      double2* nextf = i + 1 < len ? segf[i + 1] : fX;
      ABC_TRY(step_keeping(i, seg[i], nf ? segf[i] : nullptr, next, nf ? nextf : nullptr));
    }
    for (int i = len - 1; i >= 0; --i) {
      if (horner) {
        // adjoint step from lcur into lnext on the fused kernels (the aux
        // out of place: mu -> mu2), keeping its Horner increments
        ABC_TRY(launch_step_fused_keepd(La, S, lcur, nf ? mu : nullptr, lnext, nf ? mu2 : nullptr, V, ky, st));
        std::swap(mu, mu2);
        vgrad_horner2_kernel<<<gb, kBlock, 0, st>>>(
            a.grad_V, lcur, static_cast<double2*>(ky[0]), static_cast<double2*>(ky[1]), static_cast<double2*>(ky[2]),
            static_cast<double2*>(kz[3 * i]), static_cast<double2*>(kz[3 * i + 1]),
            static_cast<double2*>(kz[3 * i + 2]), seg[i], npl, L.dt);
        ABC_TRY(hipGetLastError());
        std::swap(lcur, lnext);
        continue;
      }
      // adjoint step from lcur into lnext (mu in place), keeping its stage vectors
      ABC_TRY(launch_step_staged(La, S, lnext, nf ? mu : nullptr, V, 1, st, nullptr, ky, lcur));
      vgrad_kernel<<<gb, kBlock, 0, st>>>(a.grad_V, lcur, static_cast<double2*>(ky[0]),
                                            static_cast<double2*>(ky[1]), static_cast<double2*>(ky[2]), seg[i],
                                            static_cast<double2*>(kz[3 * i]), static_cast<double2*>(kz[3 * i + 1]),
                                            static_cast<double2*>(kz[3 * i + 2]), npl, L.dt);
      ABC_TRY(hipGetLastError());
      std::swap(lcur, lnext);
    }
  }
  ABC_TRY(hipMemcpyAsync(a.grad_psi0, lcur, pb, hipMemcpyDeviceToDevice, st));
  ABC_TRY(hipMemcpyAsync(a.J_host, Jd, sizeof(double), hipMemcpyDeviceToHost, st));
  ABC_TRY(hipStreamSynchronize(st));
#undef ABC_TRY
  return ABC_OK;
}
