// Host-side setup of the boundary operators (FP64).  Not timed; runs once
// per context.  Face form: half-line DtN symbols per transverse Fourier mode
// (computed by cyclic reduction of the semi-infinite exterior operator) and
// their Fourier coefficients; box form lives in setup_box.cpp.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "abc_internal.h"

namespace abc {

Geometry make_geometry(int nx, int ny, int nz, int R, int batch) {
  Geometry g{};
  g.nx = nx; g.ny = ny; g.nz = nz; g.R = R; g.batch = batch;
  g.npts = (long long)nx * ny * nz;
  const int n1[6] = {nz, nz, nz, nz, ny, ny};
  const int n2[6] = {ny, ny, nx, nx, nx, nx};
  g.face_off[0] = 0;
  for (int f = 0; f < 6; ++f) {
    g.face_n1[f] = n1[f];
    g.face_n2[f] = n2[f];
    g.face_off[f + 1] = g.face_off[f] + (long long)R * n1[f] * n2[f] * batch;
  }
  return g;
}

// Second-derivative weights exact on polynomials of degree 2R+1 (the R = 2
// and R = 4 sets are printed in Sec. 2 / App. B and App. D).
void fd_weights(int R, double* c) {
  switch (R) {
    case 1: c[0] = -2.0; c[1] = 1.0; break;
    case 2: c[0] = -5.0 / 2; c[1] = 4.0 / 3; c[2] = -1.0 / 12; break;
    case 3: c[0] = -49.0 / 18; c[1] = 3.0 / 2; c[2] = -3.0 / 20; c[3] = 1.0 / 90; break;
    default: c[0] = 0; break;
  }
}

// ---- small dense complex helpers (n <= 3) --------------------------------

static void mat_mul(int n, const cd* A, const cd* B, cd* C) {
  cd t[kMaxR * kMaxR];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      cd s = 0;
      for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + j];
      t[i * n + j] = s;
    }
  std::memcpy(C, t, sizeof(cd) * n * n);
}

static bool mat_inv(int n, const cd* A, cd* Ainv) {
  cd a[kMaxR * kMaxR], b[kMaxR * kMaxR];
  std::memcpy(a, A, sizeof(cd) * n * n);
  for (int i = 0; i < n * n; ++i) b[i] = 0;
  for (int i = 0; i < n; ++i) b[i * n + i] = 1;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::abs(a[r * n + col]) > std::abs(a[piv * n + col])) piv = r;
    if (std::abs(a[piv * n + col]) == 0.0) return false;
    if (piv != col)
      for (int k = 0; k < n; ++k) {
        std::swap(a[piv * n + k], a[col * n + k]);
        std::swap(b[piv * n + k], b[col * n + k]);
      }
    cd d = 1.0 / a[col * n + col];
    for (int k = 0; k < n; ++k) { a[col * n + k] *= d; b[col * n + k] *= d; }
    for (int r = 0; r < n; ++r)
      if (r != col) {
        cd f = a[r * n + col];
        for (int k = 0; k < n; ++k) { a[r * n + k] -= f * a[col * n + k]; b[r * n + k] -= f * b[col * n + k]; }
      }
  }
  std::memcpy(Ainv, b, sizeof(cd) * n * n);
  return true;
}

static double mat_norm(int n, const cd* A) {
  double s = 0;
  for (int i = 0; i < n * n; ++i) s = std::max(s, std::abs(A[i]));
  return s;
}

// X Hermitian (n <= 3): true when X <= tol * I (Cholesky of tol I - X).
static bool herm_below(int n, const cd* X, double tol) {
  cd a[kMaxR * kMaxR];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) a[i * n + j] = (i == j ? cd(tol) : cd(0)) - X[i * n + j];
  for (int j = 0; j < n; ++j) {
    double d = a[j * n + j].real();
    for (int k = 0; k < j; ++k) d -= std::norm(a[j * n + k]);
    if (!(d > 0)) return false;
    double l = std::sqrt(d);
    a[j * n + j] = l;
    for (int i = j + 1; i < n; ++i) {
      cd s = a[i * n + j];
      for (int k = 0; k < j; ++k) s -= a[i * n + k] * std::conj(a[j * n + k]);
      a[i * n + j] = s / l;
    }
  }
  return true;
}

// Coupling of the R box layers (rows p) to the first R exterior points
// (columns e, x = -1 - e): -c_{p+1+e}/(2h^2) when p + 1 + e <= R.
static void face_coupling(int R, double h, double* Hgb) {
  double c[kMaxR + 1];
  fd_weights(R, c);
  for (int p = 0; p < R; ++p)
    for (int e = 0; e < R; ++e) Hgb[p * R + e] = (p + 1 + e <= R) ? -c[p + 1 + e] / (2 * h * h) : 0.0;
}

// The exterior x <= -1 of one normal line, ordered outward and grouped into
// blocks of R points, is block tridiagonal and block Toeplitz: diagonal D,
// coupling U to the next block out, L = U^T back.  Eliminating every second
// block repeatedly (cyclic reduction) converges quadratically to the Schur
// complement of the first block, whose inverse is the first diagonal block of
// (H_{II,II} + shift)^{-1}.  The DtN symbol is then
//   k^ = -H_{Gamma,B0} [(H_{II,II} + shift)^{-1}]_{00} H_{B0,Gamma}.
void halfline_symbol(int R, double h, cd shift, cd* out) {
  double c[kMaxR + 1];
  fd_weights(R, c);
  cd a[kMaxR + 1];
  a[0] = -c[0] / (2 * h * h) + shift;
  for (int k = 1; k <= R; ++k) a[k] = -c[k] / (2 * h * h);
  const int n = R;
  cd D[9], U[9], Lm[9];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      D[i * n + j] = a[std::abs(i - j)];
      U[i * n + j] = (j <= i) ? a[R + j - i] : cd(0);
      Lm[j * n + i] = U[i * n + j];
    }
  cd A1[9], A0[9], A2[9], Ah[9], X[9], t1[9], t2[9], tmp[9];
  std::memcpy(A1, D, sizeof(cd) * n * n);
  std::memcpy(Ah, D, sizeof(cd) * n * n);
  std::memcpy(A0, U, sizeof(cd) * n * n);
  std::memcpy(A2, Lm, sizeof(cd) * n * n);
  for (int it = 0; it < 200; ++it) {
    mat_inv(n, A1, X);
    mat_mul(n, A0, X, tmp); mat_mul(n, tmp, A2, t1);   // A0 X A2
    mat_mul(n, A2, X, tmp); mat_mul(n, tmp, A0, t2);   // A2 X A0
    for (int i = 0; i < n * n; ++i) { Ah[i] -= t1[i]; A1[i] -= t1[i] + t2[i]; }
    mat_mul(n, A0, X, tmp); mat_mul(n, tmp, A0, A0);
    mat_mul(n, A2, X, tmp); mat_mul(n, tmp, A2, A2);
    for (int i = 0; i < n * n; ++i) { A0[i] = -A0[i]; A2[i] = -A2[i]; }
    if (mat_norm(n, A0) < 1e-300 || mat_norm(n, A0) < 1e-18 * mat_norm(n, A1)) break;
  }
  cd Y[9];
  mat_inv(n, Ah, Y);
  double Hgb[9];
  face_coupling(R, h, Hgb);
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      cd s = 0;
      for (int e = 0; e < n; ++e)
        for (int f = 0; f < n; ++f) s += Hgb[p * n + e] * Y[e * n + f] * Hgb[q * n + f];
      out[p * n + q] = -s;
    }
}

static double sym1d(int R, double h, double th) {
  double c[kMaxR + 1];
  fd_weights(R, c);
  double acc = -c[0];
  for (int k = 1; k <= R; ++k) acc -= 2 * c[k] * std::cos(k * th);
  return acc / (2 * h * h);
}

static int symbol_points(double s, double h, int w) {
  double need = std::max({64.0, 4.0 * (w + 1), 60.0 / (std::sqrt(s) * h) + 2.0 * w});
  int P = 64;
  while (P < need) P *= 2;
  return P;
}

abc_status build_face_ops(const abc_params& p, FaceOps& ops, std::string& err) {
  const int R = p.radius, w = p.window, n = R;
  const double h = p.h;
  const bool first = p.order == ABC_FIRST;
  const double s = first ? p.s1 : p.s0;
  if (!(s > 0)) { err = "interpolation point must be positive"; return ABC_EUNSTABLE; }
  ops.R = R;
  ops.w = w;
  const int P = symbol_points(s, h, w);
  const int H = P / 2;  // theta_j = 2 pi j / P, j = 0..H covers [0, pi]
  std::vector<double> th(H + 1), tau1(H + 1), mult(H + 1);
  for (int j = 0; j <= H; ++j) {
    th[j] = 2 * M_PI * j / P;
    tau1[j] = sym1d(R, h, th[j]);
    mult[j] = (j == 0 || j == H) ? 1.0 : 2.0;
  }
  double Hgb[9], HH[9];
  face_coupling(R, h, Hgb);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double sacc = 0;
      for (int e = 0; e < n; ++e) sacc += Hgb[i * n + e] * Hgb[j * n + e];
      HH[i * n + j] = sacc;
    }
  cd HHc[9], Qc[9];
  for (int i = 0; i < n * n; ++i) { HHc[i] = HH[i]; ops.a[i] = cd(0, -1) * HH[i]; }
  mat_inv(n, HHc, Qc);
  for (int i = 0; i < n * n; ++i) ops.q[i] = Qc[i];

  // Lyapunov weight q = Lc Lc^T: in the coordinates g = Lc^T f the first-order
  // operator is Lc^T B Lc^{-T}; its norm bounds the boundary spectrum
  double Lc[9] = {0};
  for (int j = 0; j < n; ++j) {
    double d = Qc[j * n + j].real();
    for (int k = 0; k < j; ++k) d -= Lc[j * n + k] * Lc[j * n + k];
    Lc[j * n + j] = std::sqrt(std::max(d, 1e-300));
    for (int i = j + 1; i < n; ++i) {
      double v = Qc[i * n + j].real();
      for (int k = 0; k < j; ++k) v -= Lc[i * n + k] * Lc[j * n + k];
      Lc[i * n + j] = v / Lc[j * n + j];
    }
  }
  cd LcT[9], LcTinv[9];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) LcT[i * n + j] = Lc[j * n + i];
  mat_inv(n, LcT, LcTinv);
  double cn = 0;
  for (int i = 0; i < n * n; ++i) cn += Hgb[i] * Hgb[i];
  ops.coupling_norm = std::sqrt(cn);
  double symnorm = 0;

  // symbol on the quarter grid, with the sign condition of the relevant
  // stability theorem checked mode by mode
  std::vector<cd> sym((size_t)(H + 1) * (H + 1) * n * n);
  for (int j1 = 0; j1 <= H; ++j1)
    for (int j2 = 0; j2 <= j1; ++j2) {
      cd k[9], out[9];
      halfline_symbol(R, h, cd(tau1[j1] + tau1[j2], -s), k);
      if (!first) {
        std::memcpy(out, k, sizeof(cd) * n * n);
        cd im[9];
        for (int a = 0; a < n; ++a)
          for (int b = 0; b < n; ++b) im[a * n + b] = (k[a * n + b] - std::conj(k[b * n + a])) / cd(0, 2);
        if (!herm_below(n, im, 1e-12 * mat_norm(n, k))) {
          err = "zeroth-order symbol has Im K not negative semidefinite";
          return ABC_EUNSTABLE;
        }
      } else {
        cd kinv[9], akinv[9];
        if (!mat_inv(n, k, kinv)) { err = "singular half-line symbol"; return ABC_EUNSTABLE; }
        mat_mul(n, ops.a, kinv, akinv);
        for (int a = 0; a < n; ++a)
          for (int b = 0; b < n; ++b) out[a * n + b] = (a == b ? cd(s) : cd(0)) - akinv[a * n + b];
        cd qb[9], hq[9];
        mat_mul(n, ops.q, out, qb);
        for (int a = 0; a < n; ++a)
          for (int b = 0; b < n; ++b) hq[a * n + b] = 0.5 * (qb[a * n + b] + std::conj(qb[b * n + a]));
        if (!herm_below(n, hq, 1e-11 * mat_norm(n, qb))) {
          err = "first-order symbol has Q B + B^* Q not negative semidefinite";
          return ABC_EUNSTABLE;
        }
      }
      {
        cd t[9], u[9];
        if (first) {
          mat_mul(n, LcT, out, t);
          mat_mul(n, t, LcTinv, u);
        } else {
          std::memcpy(u, out, sizeof(cd) * n * n);
        }
        double fr = 0;
        for (int i = 0; i < n * n; ++i) fr += std::norm(u[i]);
        symnorm = std::max(symnorm, std::sqrt(fr));
      }
      for (int i = 0; i < n * n; ++i) {
        sym[((size_t)j1 * (H + 1) + j2) * n * n + i] = out[i];
        sym[((size_t)j2 * (H + 1) + j1) * n * n + i] = out[i];
      }
    }
  // Fourier coefficients k(p) = P^-2 sum_theta k^(theta) e^{i p.theta}; the
  // symbol is even in each angle, so this is a separable cosine sum.
  const int W = w + 1;
  std::vector<double> cosv((size_t)(H + 1) * W);
  for (int j = 0; j <= H; ++j)
    for (int q = 0; q < W; ++q) cosv[(size_t)j * W + q] = std::cos(q * th[j]);
  std::vector<cd> S((size_t)(H + 1) * W * n * n, cd(0));
  for (int j1 = 0; j1 <= H; ++j1)
    for (int j2 = 0; j2 <= H; ++j2) {
      const cd* sv = &sym[((size_t)j1 * (H + 1) + j2) * n * n];
      for (int q = 0; q < W; ++q) {
        double f = mult[j2] * cosv[(size_t)j2 * W + q];
        cd* dst = &S[((size_t)j1 * W + q) * n * n];
        for (int i = 0; i < n * n; ++i) dst[i] += f * sv[i];
      }
    }
  const int K = 2 * w + 1;
  ops.kernel.assign((size_t)n * n * K * K, cd(0));
  const double inv = 1.0 / ((double)P * P);
  for (int p1 = 0; p1 < W; ++p1)
    for (int p2 = 0; p2 < W; ++p2) {
      cd acc[9] = {};
      for (int j1 = 0; j1 <= H; ++j1) {
        double f = mult[j1] * cosv[(size_t)j1 * W + p1];
        const cd* sv = &S[((size_t)j1 * W + p2) * n * n];
        for (int i = 0; i < n * n; ++i) acc[i] += f * sv[i];
      }
      double win = 1.0;
      if (p.fejer) win = (1.0 - p1 / (double)(w + 1)) * (1.0 - p2 / (double)(w + 1));
      for (int sg1 = -1; sg1 <= 1; sg1 += 2)
        for (int sg2 = -1; sg2 <= 1; sg2 += 2) {
          int i1 = sg1 * p1 + w, i2 = sg2 * p2 + w;
          for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b)
              ops.kernel[(((size_t)a * n + b) * K + i1) * K + i2] = acc[a * n + b] * inv * win;
        }
    }
  double kabs = 0;
  for (int a = 0; a < n; ++a) {
    double rs = 0;
    for (int b = 0; b < n; ++b)
      for (int i = 0; i < K * K; ++i) rs += std::abs(ops.kernel[((size_t)a * n + b) * K * K + i]);
    kabs = std::max(kabs, rs);
  }
  ops.kernel_abs_sum = kabs;
  // the Fejer-smoothed symbol is a convex average of symbol values and the
  // full section sees the exact kernel, so sup |symbol| bounds both; a plain
  // truncation is bounded by the kernel's absolute sum instead
  const int nmax = std::max({p.nx, p.ny, p.nz});
  ops.symbol_norm = (p.fejer || w >= nmax - 1) ? symnorm : std::max(symnorm, kabs);
  return ABC_OK;
}

}  // namespace abc
