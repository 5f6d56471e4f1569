// Box form of the boundary operators: the paper's dense DtN map on Gamma.
//
//   K(s) = -(I - H_{Gamma,Sigma} G~_{Sigma,Gamma})^{-1} H_{Gamma,Sigma} G~_{Sigma,Sigma} H_{Sigma,Gamma}
//
// (App. A), with G~ the lattice Green's function of H - i s on Z^3 (App. D),
// evaluated as the Brillouin-zone integral by the trapezoidal rule on an
// L-periodic lattice (an inverse 3D FFT written here).  The dense solves run
// on the device through rocSOLVER (setup only, never on the stepping path).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "abc_internal.h"

namespace abc {
namespace {

// in-place iterative radix-2 FFT (inverse, unnormalised) on a strided line
void fft_line(cd* a, int n, long long stride, const std::vector<cd>& tw, std::vector<cd>& buf) {
  for (int i = 0; i < n; ++i) buf[i] = a[i * stride];
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(buf[i], buf[j]);
  }
  for (int len = 2; len <= n; len <<= 1) {
    const int step = n / len;
    for (int i = 0; i < n; i += len)
      for (int k = 0; k < len / 2; ++k) {
        const cd w = tw[k * step];
        const cd u = buf[i + k], v = buf[i + k + len / 2] * w;
        buf[i + k] = u + v;
        buf[i + k + len / 2] = u - v;
      }
  }
  for (int i = 0; i < n; ++i) a[i * stride] = buf[i];
}

void ifft3(std::vector<cd>& a, int L) {
  std::vector<cd> tw(L);
  for (int k = 0; k < L; ++k) tw[k] = std::polar(1.0, 2 * M_PI * k / L);  // e^{+i...}: inverse
  const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  for (int axis = 0; axis < 3; ++axis) {
    const long long stride = axis == 0 ? 1LL : (axis == 1 ? (long long)L : (long long)L * L);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
      th.emplace_back([&, t]() {
        std::vector<cd> buf(L);
        for (long long line = t; line < (long long)L * L; line += nt) {
          const long long u = line % L, v = line / L;
          long long base;
          if (axis == 0) base = (v * L + u) * L;
          else if (axis == 1) base = v * L * L + u;
          else base = v * L + u;
          fft_line(a.data() + base, L, stride, tw, buf);
        }
      });
    for (auto& t : th) t.join();
  }
  const double inv = 1.0 / ((double)L * L * L);
  for (auto& x : a) x *= inv;
}

struct Coupled {
  int q[3 * kMaxR * 3][3];  // exterior neighbours (z, y, x)
  double w[3 * kMaxR * 3];
  int n = 0;
};

struct BoxGeom {
  int nx, ny, nz, R;
  std::vector<int> glin;            // gamma -> linear index
  std::vector<int> gz, gy, gx;
  std::vector<Coupled> cpl;         // per gamma point: couplings to Sigma
};

BoxGeom box_geometry(const abc_params& p) {
  BoxGeom b;
  b.nx = p.nx; b.ny = p.ny; b.nz = p.nz; b.R = p.radius;
  double c[kMaxR + 1];
  fd_weights(p.radius, c);
  const int R = p.radius;
  for (int z = 0; z < p.nz; ++z)
    for (int y = 0; y < p.ny; ++y)
      for (int x = 0; x < p.nx; ++x) {
        const bool in = x < R || x >= p.nx - R || y < R || y >= p.ny - R || z < R || z >= p.nz - R;
        if (!in) continue;
        b.glin.push_back((z * p.ny + y) * p.nx + x);
        b.gz.push_back(z); b.gy.push_back(y); b.gx.push_back(x);
        Coupled cp;
        const int pt[3] = {z, y, x};
        const int dims[3] = {p.nz, p.ny, p.nx};
        for (int a = 0; a < 3; ++a)
          for (int k = -R; k <= R; ++k) {
            if (k == 0) continue;
            int q[3] = {pt[0], pt[1], pt[2]};
            q[a] += k;
            if (q[a] >= 0 && q[a] < dims[a]) continue;
            cp.q[cp.n][0] = q[0]; cp.q[cp.n][1] = q[1]; cp.q[cp.n][2] = q[2];
            cp.w[cp.n] = -c[std::abs(k)] / (2 * p.h * p.h);
            ++cp.n;
          }
        b.cpl.push_back(cp);
      }
  return b;
}

int lattice_size(const abc_params& p, double s) {
  const int nmax = std::max({p.nx, p.ny, p.nz});
  const double need = 2.0 * (nmax + 2 * p.radius) + std::ceil(35.0 / (std::sqrt(s) * p.h));
  int L = 16;
  while (L < need) L *= 2;
  return L;
}

// K(s) in column-major order (n x n), host
abc_status dtn_matrix(const abc_params& p, const BoxGeom& bg, double s, rocblas_handle hnd, std::vector<cd>& Kcm,
                      std::string& err) {
  const int L = lattice_size(p, s);
  if ((double)L * L * L * 16 > 4.5e9) { err = "lattice Green's function table too large"; return ABC_ENOMEM; }
  double c[kMaxR + 1];
  fd_weights(p.radius, c);
  std::vector<double> s1(L);
  for (int j = 0; j < L; ++j) {
    const double th = 2 * M_PI * j / L;
    double acc = -c[0];
    for (int k = 1; k <= p.radius; ++k) acc -= 2 * c[k] * std::cos(k * th);
    s1[j] = acc / (2 * p.h * p.h);
  }
  std::vector<cd> G((size_t)L * L * L);
  for (int i = 0; i < L; ++i)
    for (int j = 0; j < L; ++j)
      for (int k = 0; k < L; ++k) G[((size_t)i * L + j) * L + k] = 1.0 / cd(s1[i] + s1[j] + s1[k], -s);
  ifft3(G, L);
  auto Gat = [&](int dz, int dy, int dx) {
    dz = ((dz % L) + L) % L; dy = ((dy % L) + L) % L; dx = ((dx % L) + L) % L;
    return G[((size_t)dz * L + dy) * L + dx];
  };
  const int n = (int)bg.glin.size();
  // ImT = I - H_gs G_sg  and  S = H_gs G_ss H_sg, both column-major
  std::vector<cd> A((size_t)n * n), S((size_t)n * n);
  const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&, t]() {
      for (int j = t; j < n; j += nt) {
        const Coupled& cj = bg.cpl[j];
        for (int i = 0; i < n; ++i) {
          const Coupled& ci = bg.cpl[i];
          cd tv = 0, sv = 0;
          for (int a = 0; a < ci.n; ++a) {
            tv += ci.w[a] * Gat(ci.q[a][0] - bg.gz[j], ci.q[a][1] - bg.gy[j], ci.q[a][2] - bg.gx[j]);
            for (int b2 = 0; b2 < cj.n; ++b2)
              sv += ci.w[a] * cj.w[b2] *
                    Gat(ci.q[a][0] - cj.q[b2][0], ci.q[a][1] - cj.q[b2][1], ci.q[a][2] - cj.q[b2][2]);
          }
          A[(size_t)j * n + i] = (i == j ? cd(1) : cd(0)) - tv;
          S[(size_t)j * n + i] = sv;
        }
      }
    });
  for (auto& x : th) x.join();
  G.clear();
  G.shrink_to_fit();
  // solve (I - T) X = S on the device; K = -X
  rocblas_double_complex *dA = nullptr, *dB = nullptr;
  rocblas_int *ipiv = nullptr, *info = nullptr;
  const size_t bytes = (size_t)n * n * sizeof(rocblas_double_complex);
  if (hipMalloc(&dA, bytes) != hipSuccess || hipMalloc(&dB, bytes) != hipSuccess ||
      hipMalloc(&ipiv, n * sizeof(rocblas_int)) != hipSuccess || hipMalloc(&info, sizeof(rocblas_int)) != hipSuccess) {
    (void)hipFree(dA); (void)hipFree(dB); (void)hipFree(ipiv); (void)hipFree(info);
    err = "device allocation for the DtN solve failed";
    return ABC_ENOMEM;
  }
  abc_status st = ABC_OK;
  rocblas_int hinfo = 0;
  if (hipMemcpy(dA, A.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dB, S.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
    err = "hipMemcpy failed"; st = ABC_EDEVICE;
  } else if (rocsolver_zgetrf(hnd, n, n, dA, n, ipiv, info) != rocblas_status_success ||
             rocsolver_zgetrs(hnd, rocblas_operation_none, n, n, dA, n, ipiv, dB, n) != rocblas_status_success) {
    err = "rocSOLVER failed"; st = ABC_EDEVICE;
  } else if (hipMemcpy(&hinfo, info, sizeof(rocblas_int), hipMemcpyDeviceToHost) != hipSuccess || hinfo != 0) {
    err = "I - H G is singular"; st = ABC_EUNSTABLE;
  } else {
    Kcm.resize((size_t)n * n);
    if (hipMemcpy(Kcm.data(), dB, bytes, hipMemcpyDeviceToHost) != hipSuccess) { err = "hipMemcpy failed"; st = ABC_EDEVICE; }
    for (auto& x : Kcm) x = -x;
  }
  (void)hipFree(dA); (void)hipFree(dB); (void)hipFree(ipiv); (void)hipFree(info);
  return st;
}

// X = A^{-1} B for column-major n x n host matrices (device solve)
abc_status solve_cm(rocblas_handle hnd, int n, const std::vector<cd>& A, const std::vector<cd>& B, std::vector<cd>& X,
                    std::string& err) {
  rocblas_double_complex *dA = nullptr, *dB = nullptr;
  rocblas_int *ipiv = nullptr, *info = nullptr;
  const size_t bytes = (size_t)n * n * sizeof(rocblas_double_complex);
  if (hipMalloc(&dA, bytes) != hipSuccess || hipMalloc(&dB, bytes) != hipSuccess ||
      hipMalloc(&ipiv, n * sizeof(rocblas_int)) != hipSuccess || hipMalloc(&info, sizeof(rocblas_int)) != hipSuccess) {
    (void)hipFree(dA); (void)hipFree(dB); (void)hipFree(ipiv); (void)hipFree(info);
    err = "device allocation failed";
    return ABC_ENOMEM;
  }
  abc_status st = ABC_OK;
  rocblas_int hinfo = 0;
  if (hipMemcpy(dA, A.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dB, B.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
    err = "hipMemcpy failed"; st = ABC_EDEVICE;
  } else if (rocsolver_zgetrf(hnd, n, n, dA, n, ipiv, info) != rocblas_status_success ||
             rocsolver_zgetrs(hnd, rocblas_operation_none, n, n, dA, n, ipiv, dB, n) != rocblas_status_success) {
    err = "rocSOLVER failed"; st = ABC_EDEVICE;
  } else if (hipMemcpy(&hinfo, info, sizeof(rocblas_int), hipMemcpyDeviceToHost) != hipSuccess || hinfo != 0) {
    err = "singular matrix in the first-order construction"; st = ABC_EUNSTABLE;
  } else {
    X.resize((size_t)n * n);
    if (hipMemcpy(X.data(), dB, bytes, hipMemcpyDeviceToHost) != hipSuccess) { err = "hipMemcpy failed"; st = ABC_EDEVICE; }
  }
  (void)hipFree(dA); (void)hipFree(dB); (void)hipFree(ipiv); (void)hipFree(info);
  return st;
}

}  // namespace

abc_status build_box_ops(const abc_params& p, double2** mat_dev, double2** q_dev, int* n_gamma,
                         std::vector<int>& gamma_lin, double* spectral_bound, std::string& err) {
  *mat_dev = nullptr;
  *q_dev = nullptr;
  BoxGeom bg = box_geometry(p);
  const int n = (int)bg.glin.size();
  *n_gamma = n;
  gamma_lin = bg.glin;
  if ((double)n * n * 16 * 6 > 200e9) { err = "box form too large for this box; use the face form"; return ABC_ENOMEM; }
  rocblas_handle hnd;
  if (rocblas_create_handle(&hnd) != rocblas_status_success) { err = "rocblas_create_handle failed"; return ABC_EDEVICE; }
  abc_status st = ABC_OK;
  const bool first = p.order == ABC_FIRST;
  std::vector<cd> out_rm;  // row-major result uploaded to the device
  std::vector<cd> Qrm;
  double bound = 0;
  if (!first) {
    std::vector<cd> K;
    st = dtn_matrix(p, bg, p.s0, hnd, K, err);
    if (st == ABC_OK) {
      out_rm.resize((size_t)n * n);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) out_rm[(size_t)i * n + j] = K[(size_t)j * n + i];
    }
  } else {
    // H_{Gamma,II} H_{II,Gamma}: entries couple Gamma points sharing a Sigma point
    std::vector<cd> HH((size_t)n * n, cd(0));
    {
      // index Sigma points
      std::vector<std::pair<long long, std::pair<int, double>>> lst;
      for (int i = 0; i < n; ++i)
        for (int a = 0; a < bg.cpl[i].n; ++a) {
          const int* q = bg.cpl[i].q[a];
          const long long key = (((long long)(q[0] + 8)) * 4096 + (q[1] + 8)) * 4096 + (q[2] + 8);
          lst.push_back({key, {i, bg.cpl[i].w[a]}});
        }
      std::sort(lst.begin(), lst.end());
      size_t a = 0;
      while (a < lst.size()) {
        size_t b2 = a;
        while (b2 < lst.size() && lst[b2].first == lst[a].first) ++b2;
        for (size_t u = a; u < b2; ++u)
          for (size_t v = a; v < b2; ++v)
            HH[(size_t)lst[u].second.first * n + lst[v].second.first] += lst[u].second.second * lst[v].second.second;
        a = b2;
      }
    }
    std::vector<cd> K1;
    st = dtn_matrix(p, bg, p.s1, hnd, K1, err);
    std::vector<cd> Bcm, Acm;
    if (st == ABC_OK && !(p.s2 > 0)) {
      // theorem pair: A = -i HH, B = s1 I - A K1^{-1} = s1 I - (K1^{-1} A)^T
      Acm.resize((size_t)n * n);
      for (size_t i = 0; i < Acm.size(); ++i) Acm[i] = cd(0, -1) * HH[i];  // HH symmetric: layout-free
      std::vector<cd> X;
      st = solve_cm(hnd, n, K1, Acm, X, err);
      if (st == ABC_OK) {
        Bcm.resize((size_t)n * n);
        // B = s1 I - X^T ; column-major B[j*n+i] = B_ij = s1 d_ij - X_ji = s1 d_ij - Xcm[i*n+j]
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) Bcm[(size_t)j * n + i] = (i == j ? cd(p.s1) : cd(0)) - X[(size_t)i * n + j];
      }
    } else if (st == ABC_OK) {
      std::vector<cd> K2;
      st = dtn_matrix(p, bg, p.s2, hnd, K2, err);
      if (st == ABC_OK) {
        // (K2 - K1) B^T = s2 K2 - s1 K1  (K symmetric)
        std::vector<cd> D((size_t)n * n), Rh((size_t)n * n), BT;
        for (size_t i = 0; i < D.size(); ++i) { D[i] = K2[i] - K1[i]; Rh[i] = p.s2 * K2[i] - p.s1 * K1[i]; }
        st = solve_cm(hnd, n, D, Rh, BT, err);
        if (st == ABC_OK) {
          Bcm.resize((size_t)n * n);
          for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) Bcm[(size_t)j * n + i] = BT[(size_t)i * n + j];
          // A = (s1 I - B) K1 = s1 K1 - B K1 (device GEMM)
          Acm.resize((size_t)n * n);
          rocblas_double_complex *dB = nullptr, *dK = nullptr, *dC = nullptr;
          const size_t bytes = (size_t)n * n * 16;
          if (hipMalloc(&dB, bytes) != hipSuccess || hipMalloc(&dK, bytes) != hipSuccess ||
              hipMalloc(&dC, bytes) != hipSuccess) {
            err = "hipMalloc failed"; st = ABC_ENOMEM;
          } else {
            const rocblas_double_complex alpha(-1.0, 0.0), beta(p.s1, 0.0);
            if (hipMemcpy(dB, Bcm.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(dK, K1.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(dC, K1.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
                rocblas_zgemm(hnd, rocblas_operation_none, rocblas_operation_none, n, n, n, &alpha, dB, n, dK, n,
                              &beta, dC, n) != rocblas_status_success ||
                hipMemcpy(Acm.data(), dC, bytes, hipMemcpyDeviceToHost) != hipSuccess) {
              err = "device GEMM for A failed"; st = ABC_EDEVICE;
            }
          }
          (void)hipFree(dB); (void)hipFree(dK); (void)hipFree(dC);
        }
      }
    }
    if (st == ABC_OK) {
      out_rm.resize((size_t)n * 2 * n);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          out_rm[(size_t)i * 2 * n + j] = Bcm[(size_t)j * n + i];
          out_rm[(size_t)i * 2 * n + n + j] = Acm[(size_t)j * n + i];
        }
      // Q = HH^{-1}
      std::vector<cd> I((size_t)n * n, cd(0)), Qcm;
      for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1;
      st = solve_cm(hnd, n, HH, I, Qcm, err);
      if (st == ABC_OK) {
        Qrm.resize((size_t)n * n);
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) Qrm[(size_t)i * n + j] = Qcm[(size_t)j * n + i];
      }
    }
  }
  rocblas_destroy_handle(hnd);
  if (st != ABC_OK) return st;
  // spectral radius of M (zeroth) or B (first) by power iteration, with a
  // safety factor; the row-sum norm of these dense non-normal matrices is far
  // above their spectral radius
  {
    const int ncol = first ? 2 * n : n;
    std::vector<cd> v(n), u(n);
    for (int i = 0; i < n; ++i) v[i] = cd(std::cos(0.7 * i + 0.1), std::sin(1.3 * i));
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    double est = 0;
    for (int it = 0; it < 60; ++it) {
      std::vector<std::thread> th;
      for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
          for (int i = t; i < n; i += nt) {
            cd acc = 0;
            const cd* row = &out_rm[(size_t)i * ncol];
            for (int j = 0; j < n; ++j) acc += row[j] * v[j];
            u[i] = acc;
          }
        });
      for (auto& x : th) x.join();
      double nu = 0, nv = 0;
      for (int i = 0; i < n; ++i) { nu += std::norm(u[i]); nv += std::norm(v[i]); }
      est = std::sqrt(nu / nv);
      const double sc = 1.0 / std::sqrt(nu);
      for (int i = 0; i < n; ++i) v[i] = u[i] * sc;
    }
    bound = 1.25 * est;
  }
  *spectral_bound = bound;
  void* d = nullptr;
  if (hipMalloc(&d, out_rm.size() * 16) != hipSuccess) { err = "hipMalloc of box operator failed"; return ABC_ENOMEM; }
  if (hipMemcpy(d, out_rm.data(), out_rm.size() * 16, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    err = "hipMemcpy failed";
    return ABC_EDEVICE;
  }
  *mat_dev = static_cast<double2*>(d);
  if (first) {
    void* qd = nullptr;
    if (hipMalloc(&qd, Qrm.size() * 16) != hipSuccess ||
        hipMemcpy(qd, Qrm.data(), Qrm.size() * 16, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(qd);
      (void)hipFree(d);
      *mat_dev = nullptr;
      err = "upload of Q failed";
      return ABC_EDEVICE;
    }
    *q_dev = static_cast<double2*>(qd);
  }
  return ABC_OK;
}

}  // namespace abc
