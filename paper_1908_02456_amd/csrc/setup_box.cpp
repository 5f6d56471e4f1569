// Box form of the boundary operators: the paper's dense DtN map on Gamma,
//
//   K(s) = -(I - H_{Gamma,Sigma} G~_{Sigma,Gamma})^{-1} H_{Gamma,Sigma} G~_{Sigma,Sigma} H_{Sigma,Gamma}
//
// (App. A), with G~ the lattice Green's function of H - i s on Z^3 (App. D)
// evaluated as the Brillouin-zone integral by the trapezoidal rule on an
// L-periodic lattice, i.e. an inverse 3D FFT of the symbol.  Everything of
// size n_Gamma^2 or L^3 is built on the device: the symbol table and its FFT
// (LDS line transforms written here), the assembly of I - T and -S from the
// table, the dense LU solves (rocSOLVER), the order-specific products
// (rocBLAS) and layout changes, and the power-iteration bound.  The host
// only builds the geometry of Gamma and its couplings to Sigma.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

#include "abc_internal.h"

namespace abc {
namespace {

constexpr int kMaxCpl = 3 * kMaxR;  // exterior neighbours of one Gamma point
constexpr int kThreads = 256;

struct BoxGeom {
  int nx, ny, nz, R;
  std::vector<int> glin;            // gamma -> linear index
  std::vector<int> pos;             // gamma -> (z, y, x)
  std::vector<int> cnt;             // gamma -> number of Sigma couplings
  std::vector<int> cq;              // [gamma][kMaxCpl][3] Sigma points (z, y, x)
  std::vector<double> cw;           // [gamma][kMaxCpl] coupling weights
};

BoxGeom box_geometry(const abc_params& p) {
  BoxGeom b;
  b.nx = p.nx; b.ny = p.ny; b.nz = p.nz; b.R = p.radius;
  double c[kMaxR + 1];
  fd_weights(p.radius, c);
  const int R = p.radius;
  const int dims[3] = {p.nz, p.ny, p.nx};
  for (int z = 0; z < p.nz; ++z)
    for (int y = 0; y < p.ny; ++y)
      for (int x = 0; x < p.nx; ++x) {
        const bool in = x < R || x >= p.nx - R || y < R || y >= p.ny - R || z < R || z >= p.nz - R;
        if (!in) continue;
        b.glin.push_back((z * p.ny + y) * p.nx + x);
        const int pt[3] = {z, y, x};
        b.pos.insert(b.pos.end(), pt, pt + 3);
        int n = 0;
        std::vector<int> q(kMaxCpl * 3, 0);
        std::vector<double> w(kMaxCpl, 0.0);
        for (int a = 0; a < 3; ++a)
          for (int k = -R; k <= R; ++k) {
            if (k == 0) continue;
            int qq[3] = {pt[0], pt[1], pt[2]};
            qq[a] += k;
            if (qq[a] >= 0 && qq[a] < dims[a]) continue;
            q[n * 3 + 0] = qq[0]; q[n * 3 + 1] = qq[1]; q[n * 3 + 2] = qq[2];
            w[n] = -c[std::abs(k)] / (2 * p.h * p.h);
            ++n;
          }
        b.cnt.push_back(n);
        b.cq.insert(b.cq.end(), q.begin(), q.end());
        b.cw.insert(b.cw.end(), w.begin(), w.end());
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

// ---------------------------------------------------------------------------
// device kernels
// ---------------------------------------------------------------------------

// symbol of H - i s on the L-periodic lattice, divided by L^3 (the inverse
// FFT below is unnormalised): 1 / (L^3 (sig[k1] + sig[k2] + sig[k3] - i s))
__global__ void __launch_bounds__(kThreads) gf_symbol_kernel(double2* __restrict__ G, const double* __restrict__ sig,
                                                             int L, double s, double inv_vol) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)L * L * L;
  if (e >= tot) return;
  const int k3 = (int)(e % L), k2 = (int)((e / L) % L), k1 = (int)(e / ((long long)L * L));
  const double a = sig[k1] + sig[k2] + sig[k3];
  const double d = inv_vol / (a * a + s * s);  // 1/(a - i s) = (a + i s)/(a^2 + s^2)
  G[e] = make_double2(a * d, s * d);
}

// Inverse radix-2 FFT of TW lines of length L = 2^logL per workgroup, held in
// LDS as [t][k].  Line t of group g starts at a_idx * A + b_idx * TW * C + t *
// tstride (g = a_idx * (L / TW) + b_idx) and steps kstride; the three axes of
// an L^3 table are (A, C, tstride, kstride) = (L^2, L, L, 1), (L^2, 1, 1, L)
// and (L, 1, 1, L^2).  tw[k] = exp(2 pi i k / L), k < L/2.
__global__ void __launch_bounds__(kThreads) fft_lines_kernel(double2* __restrict__ a, const double2* __restrict__ tw,
                                                             int L, int logL, int TW, long long A, long long C,
                                                             long long tstride, long long kstride) {
  extern __shared__ double2 buf[];
  const int g = blockIdx.x;
  const int per = L / TW;
  const long long base = (long long)(g / per) * A + (long long)(g % per) * TW * C;
  const int tot = TW * L;
  const bool kfast = kstride == 1;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int t = kfast ? e / L : e % TW;
    const int k = kfast ? e % L : e / TW;
    const unsigned rk = __brev((unsigned)k) >> (32 - logL);
    buf[t * L + rk] = a[base + t * tstride + k * kstride];
  }
  __syncthreads();
  for (int len = 2, lshift = 1; len <= L; len <<= 1, ++lshift) {
    const int half = len >> 1;
    const int step = L >> lshift;  // twiddle stride
    for (int bf = threadIdx.x; bf < tot / 2; bf += blockDim.x) {
      const int t = bf / (L / 2), r = bf % (L / 2);
      const int grp = r / half, pos = r % half;
      const int i0 = t * L + grp * len + pos, i1 = i0 + half;
      const double2 w = tw[pos * step];
      const double2 u = buf[i0], v0 = buf[i1];
      const double2 v = make_double2(v0.x * w.x - v0.y * w.y, v0.x * w.y + v0.y * w.x);
      buf[i0] = make_double2(u.x + v.x, u.y + v.y);
      buf[i1] = make_double2(u.x - v.x, u.y - v.y);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int t = kfast ? e / L : e % TW;
    const int k = kfast ? e % L : e / TW;
    a[base + t * tstride + k * kstride] = buf[t * L + k];
  }
}

__device__ __forceinline__ double2 gf_at(const double2* __restrict__ G, int L, int dz, int dy, int dx) {
  const int m = L - 1;  // L is a power of two: & m is the periodic wrap
  return G[((long long)(dz & m) * L + (dy & m)) * L + (dx & m)];
}

// column-major n x n: ImT(i, j) = delta_ij - sum_a w_ia G(q_ia - p_j),
// negS(i, j) = -sum_a sum_b w_ia w_jb G(q_ia - q_jb)
__global__ void __launch_bounds__(kThreads) dtn_assemble_kernel(double2* __restrict__ ImT, double2* __restrict__ negS,
                                                                int n, const int* __restrict__ cnt,
                                                                const int* __restrict__ cq,
                                                                const double* __restrict__ cw,
                                                                const int* __restrict__ pos,
                                                                const double2* __restrict__ G, int L) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ni = cnt[i];
  for (int j = blockIdx.y; j < n; j += gridDim.y) {
    const int nj = cnt[j];
    const int pz = pos[3 * j], py = pos[3 * j + 1], px = pos[3 * j + 2];
    double tr = 0, ti = 0, sr = 0, si = 0;
    for (int a = 0; a < ni; ++a) {
      const int* qa = cq + ((long long)i * kMaxCpl + a) * 3;
      const double wa = cw[(long long)i * kMaxCpl + a];
      const double2 g = gf_at(G, L, qa[0] - pz, qa[1] - py, qa[2] - px);
      tr += wa * g.x;
      ti += wa * g.y;
      for (int b = 0; b < nj; ++b) {
        const int* qb = cq + ((long long)j * kMaxCpl + b) * 3;
        const double ww = wa * cw[(long long)j * kMaxCpl + b];
        const double2 g2 = gf_at(G, L, qa[0] - qb[0], qa[1] - qb[1], qa[2] - qb[2]);
        sr += ww * g2.x;
        si += ww * g2.y;
      }
    }
    const long long e = (long long)j * n + i;
    ImT[e] = make_double2((i == j ? 1.0 : 0.0) - tr, -ti);
    negS[e] = make_double2(-sr, -si);
  }
}

// dst(r, c) = alpha * M(r, c) + diag * delta_rc for r < rows, c < cols, where
// dst is row-major (dst[r * ldd + c]) and M is column-major in src
// (src[c * lds + r]): a layout change, tiled through LDS
__global__ void __launch_bounds__(kThreads) to_row_major_kernel(double2* __restrict__ dst, long long ldd,
                                                                const double2* __restrict__ src, long long lds,
                                                                int rows, int cols, double2 alpha, double diag) {
  __shared__ double2 tile[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;  // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + tx, c = c0 + k;
    if (r < rows && c < cols) tile[k][tx] = src[(long long)c * lds + r];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    if (r < rows && c < cols) {
      const double2 m = tile[tx][k];
      double2 o = make_double2(alpha.x * m.x - alpha.y * m.y, alpha.x * m.y + alpha.y * m.x);
      if (r == c) o.x += diag;
      dst[(long long)r * ldd + c] = o;
    }
  }
}

// dst[r * ldd + c] = alpha * src[r * lds + c] + diag * delta_rc (same layout)
__global__ void __launch_bounds__(kThreads) copy2d_kernel(double2* __restrict__ dst, long long ldd,
                                                          const double2* __restrict__ src, long long lds, int rows,
                                                          int cols, double2 alpha, double diag) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  for (int r = blockIdx.y; r < rows; r += gridDim.y) {
    const double2 m = src[(long long)r * lds + c];
    double2 o = make_double2(alpha.x * m.x - alpha.y * m.y, alpha.x * m.y + alpha.y * m.x);
    if (r == c) o.x += diag;
    dst[(long long)r * ldd + c] = o;
  }
}

// z = a x + b y elementwise (real a, b)
__global__ void __launch_bounds__(kThreads) axpby_kernel(double2* __restrict__ z, const double2* __restrict__ x,
                                                         const double2* __restrict__ y, double a, double b,
                                                         long long count) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const double2 u = x[e], v = y[e];
  z[e] = make_double2(a * u.x + b * v.x, a * u.y + b * v.y);
}

// out[e] = Re in[e]
__global__ void __launch_bounds__(kThreads) real_part_kernel(double* __restrict__ out, const double2* __restrict__ in,
                                                             long long count) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) out[e] = in[e].x;
}

// out[e] = in[e] + 0 i
__global__ void __launch_bounds__(kThreads) real_to_complex_kernel(double2* __restrict__ out,
                                                                   const double* __restrict__ in, long long count) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) out[e] = make_double2(in[e], 0.0);
}

// out (rows x cols, row-major) = in (rows x cols, column-major)
__global__ void __launch_bounds__(kThreads) transpose_real_kernel(double* __restrict__ out,
                                                                  const double* __restrict__ in, int rows, int cols) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)rows * cols) return;
  const long long i = e / cols, j = e % cols;
  out[e] = in[j * rows + i];
}

// column-major entries (i, j) = v from a host-built list of distinct entries
__global__ void __launch_bounds__(kThreads) scatter_kernel(double2* __restrict__ m, long long ld,
                                                           const int* __restrict__ ij, const double2* __restrict__ v,
                                                           int count) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  m[(long long)ij[2 * e + 1] * ld + ij[2 * e]] = v[e];
}

// Interpolation system of the second order, transposed (m = 4n rows):
// MT(j n + b, k n + a) = [s_j K_j, K_j, s_j I, I]_k (a, b) and
// RT(j n + b, a) = s_j^2 K_j(a, b), K_j column-major
struct FourK {
  const double2* K[4];
  double s[4];
};

__global__ void __launch_bounds__(kThreads) second_system_kernel(double2* __restrict__ MT, double2* __restrict__ RT,
                                                                 int n, FourK fk) {
  const long long m = 4LL * n;
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  const int j = (int)(r / n), b = (int)(r % n);
  const double sj = fk.s[j];
  const double2* Kj = fk.K[j];
  for (long long col = blockIdx.y; col < m + n; col += gridDim.y) {
    if (col < m) {
      const int k = (int)(col / n), a = (int)(col % n);
      double2 v;
      if (k < 2) {
        const double2 kab = Kj[(long long)b * n + a];
        const double f = k == 0 ? sj : 1.0;
        v = make_double2(f * kab.x, f * kab.y);
      } else {
        v = make_double2(a == b ? (k == 2 ? sj : 1.0) : 0.0, 0.0);
      }
      MT[col * m + r] = v;
    } else {
      const int a = (int)(col - m);
      const double2 kab = Kj[(long long)b * n + a];
      RT[(long long)a * m + r] = make_double2(sj * sj * kab.x, sj * sj * kab.y);
    }
  }
}

inline unsigned nblk(long long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------

// device allocations released at scope exit
struct DevBufs {
  std::vector<void*> ptrs;
  ~DevBufs() {
    for (void* q : ptrs) (void)hipFree(q);
  }
  template <typename T>
  bool alloc(T** out, size_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) return false;
    ptrs.push_back(q);
    *out = static_cast<T*>(q);
    return true;
  }
  void release(void* q) {
    auto it = std::find(ptrs.begin(), ptrs.end(), q);
    if (it != ptrs.end()) {
      (void)hipFree(q);
      ptrs.erase(it);
    }
  }
  void keep(void* q) {  // ownership passes to the caller
    auto it = std::find(ptrs.begin(), ptrs.end(), q);
    if (it != ptrs.end()) ptrs.erase(it);
  }
};

template <typename T>
abc_status upload(DevBufs& db, T** out, const std::vector<T>& h, std::string& err) {
  if (!db.alloc(out, std::max<size_t>(h.size(), 1))) { err = "hipMalloc failed"; return ABC_ENOMEM; }
  if (!h.empty() && hipMemcpy(*out, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    err = "hipMemcpy failed";
    return ABC_EDEVICE;
  }
  return ABC_OK;
}

using zc = rocblas_double_complex;

struct GammaDev {
  int n = 0;
  int* cnt = nullptr;
  int* cq = nullptr;
  double* cw = nullptr;
  int* pos = nullptr;
};

// solve A X = B in place of B (A: m x m column-major, destroyed; B: m x nrhs)
abc_status lu_solve(rocblas_handle hnd, DevBufs& db, int m, int nrhs, double2* A, double2* B, std::string& err,
                    const char* what) {
  // 64-bit index interface: m * m may exceed 2^31 (the second order's 4n system)
  int64_t* ipiv = nullptr;
  int64_t* info = nullptr;
  if (!db.alloc(&ipiv, (size_t)m) || !db.alloc(&info, 1)) { err = "hipMalloc failed"; return ABC_ENOMEM; }
  if (rocsolver_zgetrf_64(hnd, m, m, reinterpret_cast<zc*>(A), m, ipiv, info) != rocblas_status_success ||
      rocsolver_zgetrs_64(hnd, rocblas_operation_none, m, nrhs, reinterpret_cast<zc*>(A), m, ipiv,
                          reinterpret_cast<zc*>(B), m) != rocblas_status_success) {
    err = "rocSOLVER failed";
    return ABC_EDEVICE;
  }
  int64_t hinfo = 0;
  if (hipMemcpy(&hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost) != hipSuccess) {
    err = "hipMemcpy failed";
    return ABC_EDEVICE;
  }
  db.release(ipiv);
  db.release(info);
  if (hinfo != 0) {
    err = std::string("singular matrix: ") + what;
    return ABC_EUNSTABLE;
  }
  return ABC_OK;
}

// Second order at R >= 2 (Sec. 3.3, which leaves open how the coefficients
// are formed): the four maps are numerically rank-deficient, with singular
// values in two groups far apart (the outermost boundary layer's and the
// deeper layers', which reach the exterior only through the small outer
// stencil weights), and the 4n interpolation system is singular to working
// precision.  The interpolation then runs in the maps' dominant subspace:
// directions whose singular value (of the four maps together) is below
// kSecondTau of the largest are left out.
constexpr double kSecondTau = 1e-2;

// Real orthonormal basis of that subspace: the eigenvectors of
// Re sum_j K_j K_j^H whose eigenvalues exceed kSecondTau^2 times the largest
// (that span holds the real and imaginary parts of every column).  *U
// receives it as complex n x r column-major, or nullptr when r == n.
abc_status dominant_subspace(rocblas_handle hnd, DevBufs& db, int n, double2* const* K, double2** U, double** Ur,
                             int* r, std::string& err) {
  *U = nullptr;
  *Ur = nullptr;
  *r = n;
  // the eigen-solver's interface indexes the matrix with 32-bit integers
  if ((long long)n * n >= (1LL << 31)) {
    err = "second-order interpolation: n_Gamma too large for the eigen-decomposition";
    return ABC_ENOTSUP;
  }
  const size_t nsq = (size_t)n * n;
  double2* Gc = nullptr;
  double *Gr = nullptr, *D = nullptr, *E = nullptr;
  rocblas_int* info = nullptr;
  if (!db.alloc(&Gc, nsq) || !db.alloc(&Gr, nsq) || !db.alloc(&D, (size_t)n) || !db.alloc(&E, (size_t)n) ||
      !db.alloc(&info, 1)) {
    err = "hipMalloc failed";
    return ABC_ENOMEM;
  }
  const zc one(1.0, 0.0), zero(0.0, 0.0);
  for (int j = 0; j < 4; ++j)
    if (rocblas_zgemm_64(hnd, rocblas_operation_none, rocblas_operation_conjugate_transpose, n, n, n, &one,
                         reinterpret_cast<const zc*>(K[j]), n, reinterpret_cast<const zc*>(K[j]), n,
                         j ? &one : &zero, reinterpret_cast<zc*>(Gc), n) != rocblas_status_success) {
      err = "device GEMM for the maps' Gram matrix failed";
      return ABC_EDEVICE;
    }
  real_part_kernel<<<nblk((long long)nsq), kThreads>>>(Gr, Gc, (long long)nsq);
  if (hipGetLastError() != hipSuccess) { err = "setup kernel launch failed"; return ABC_EDEVICE; }
  db.release(Gc);
  // eigenvalues ascending, eigenvectors in place of Gr (column j for D[j])
  if (rocsolver_dsyevd(hnd, rocblas_evect_original, rocblas_fill_upper, n, Gr, n, D, E, info) !=
      rocblas_status_success) {
    err = "rocSOLVER eigen-decomposition failed";
    return ABC_EDEVICE;
  }
  std::vector<double> w(n);
  rocblas_int hinfo = 0;
  if (hipMemcpy(w.data(), D, (size_t)n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost) != hipSuccess) {
    err = "hipMemcpy failed";
    return ABC_EDEVICE;
  }
  if (hinfo != 0) {
    err = "eigen-decomposition of the maps' Gram matrix did not converge";
    return ABC_EDEVICE;
  }
  const double cut = kSecondTau * kSecondTau * w[n - 1];
  int keep = 0;
  for (int i = 0; i < n; ++i) keep += w[i] > cut;
  if (keep == 0) {
    err = "second-order interpolation: the DtN maps vanish";
    return ABC_EUNSTABLE;
  }
  *r = keep;
  if (keep == n) return ABC_OK;
  double2* Uc = nullptr;
  double* Ure = nullptr;
  if (!db.alloc(&Uc, (size_t)n * keep) || !db.alloc(&Ure, (size_t)n * keep)) { err = "hipMalloc failed"; return ABC_ENOMEM; }
  real_to_complex_kernel<<<nblk((long long)n * keep), kThreads>>>(Uc, Gr + (size_t)(n - keep) * n, (long long)n * keep);
  if (hipGetLastError() != hipSuccess) { err = "setup kernel launch failed"; return ABC_EDEVICE; }
  if (hipMemcpy(Ure, Gr + (size_t)(n - keep) * n, (size_t)n * keep * sizeof(double), hipMemcpyDeviceToDevice) !=
      hipSuccess) {
    err = "hipMemcpy failed";
    return ABC_EDEVICE;
  }
  *U = Uc;
  *Ur = Ure;
  return ABC_OK;
}

// K(s), column-major n x n, into a new device buffer *K
abc_status dtn_matrix(const abc_params& p, const GammaDev& gd, double s, rocblas_handle hnd, DevBufs& db,
                      double2** K, std::string& err) {
  const int L = lattice_size(p, s);
  const size_t vol = (size_t)L * L * L;
  if ((double)vol * 16 > 24e9) { err = "lattice Green's function table too large"; return ABC_ENOMEM; }
  double c[kMaxR + 1];
  fd_weights(p.radius, c);
  std::vector<double> sig(L);
  for (int j = 0; j < L; ++j) {
    const double th = 2 * M_PI * j / L;
    double acc = -c[0];
    for (int k = 1; k <= p.radius; ++k) acc -= 2 * c[k] * std::cos(k * th);
    sig[j] = acc / (2 * p.h * p.h);
  }
  std::vector<double2> tw(L / 2);
  for (int k = 0; k < L / 2; ++k) tw[k] = make_double2(std::cos(2 * M_PI * k / L), std::sin(2 * M_PI * k / L));
  double* dsig = nullptr;
  double2* dtw = nullptr;
  double2* G = nullptr;
  abc_status st = upload(db, &dsig, sig, err);
  if (st == ABC_OK) st = upload(db, &dtw, tw, err);
  if (st != ABC_OK) return st;
  if (!db.alloc(&G, vol)) { err = "device allocation of the Green's function table failed"; return ABC_ENOMEM; }
  gf_symbol_kernel<<<nblk((long long)vol), kThreads>>>(G, dsig, L, s, 1.0 / (double)vol);
  int logL = 0;
  while ((1 << logL) < L) ++logL;
  const int TW = std::min(L, 4096 / L);  // 64 KB of LDS per workgroup at most
  const long long LL = (long long)L * L;
  const long long prm[3][4] = {{LL, L, L, 1}, {LL, 1, 1, L}, {(long long)L, 1, 1, LL}};
  for (int ax = 0; ax < 3; ++ax)
    fft_lines_kernel<<<(unsigned)(LL / TW), kThreads, (size_t)TW * L * sizeof(double2)>>>(
        G, dtw, L, logL, TW, prm[ax][0], prm[ax][1], prm[ax][2], prm[ax][3]);
  const int n = gd.n;
  double2 *ImT = nullptr, *negS = nullptr;
  if (!db.alloc(&ImT, (size_t)n * n) || !db.alloc(&negS, (size_t)n * n)) {
    err = "device allocation for the DtN solve failed";
    return ABC_ENOMEM;
  }
  dim3 grid(nblk(n), (unsigned)std::min(n, 65535));
  dtn_assemble_kernel<<<grid, kThreads>>>(ImT, negS, n, gd.cnt, gd.cq, gd.cw, gd.pos, G, L);
  if (hipGetLastError() != hipSuccess) { err = "DtN assembly launch failed"; return ABC_EDEVICE; }
  db.release(G);
  db.release(dsig);
  db.release(dtw);
  // (I - T) K = -S
  st = lu_solve(hnd, db, n, n, ImT, negS, err, "I - H G");
  if (st != ABC_OK) return st;
  db.release(ImT);
  *K = negS;
  return ABC_OK;
}

abc_status launch_ok(std::string& err) {
  if (hipGetLastError() != hipSuccess) { err = "setup kernel launch failed"; return ABC_EDEVICE; }
  return ABC_OK;
}

void to_row_major(double2* dst, long long ldd, const double2* src, long long lds, int rows, int cols, double2 alpha,
                  double diag) {
  dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  to_row_major_kernel<<<grid, kThreads>>>(dst, ldd, src, lds, rows, cols, alpha, diag);
}

void copy2d(double2* dst, long long ldd, const double2* src, long long lds, int rows, int cols, double2 alpha,
            double diag) {
  dim3 grid(nblk(cols), (unsigned)std::min(rows, 65535));
  copy2d_kernel<<<grid, kThreads>>>(dst, ldd, src, lds, rows, cols, alpha, diag);
}

// H_{Gamma,II} H_{II,Gamma} as distinct (i, j, value) entries: Gamma points
// couple when they share a Sigma point
void gamma_sigma_product(const BoxGeom& bg, std::vector<int>& ij, std::vector<double2>& val) {
  const int n = (int)bg.glin.size();
  std::vector<std::pair<long long, std::pair<int, double>>> lst;
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < bg.cnt[i]; ++a) {
      const int* q = &bg.cq[((size_t)i * kMaxCpl + a) * 3];
      const long long key = (((long long)(q[0] + 8)) * 4096 + (q[1] + 8)) * 4096 + (q[2] + 8);
      lst.push_back({key, {i, bg.cw[(size_t)i * kMaxCpl + a]}});
    }
  std::sort(lst.begin(), lst.end());
  std::map<std::pair<int, int>, double> acc;
  size_t a = 0;
  while (a < lst.size()) {
    size_t b2 = a;
    while (b2 < lst.size() && lst[b2].first == lst[a].first) ++b2;
    for (size_t u = a; u < b2; ++u)
      for (size_t v = a; v < b2; ++v)
        acc[{lst[u].second.first, lst[v].second.first}] += lst[u].second.second * lst[v].second.second;
    a = b2;
  }
  for (const auto& kv : acc) {
    ij.push_back(kv.first.first);
    ij.push_back(kv.first.second);
    val.push_back(make_double2(kv.second, 0.0));
  }
}

// spectral radius of the leading m x m block of the row-major operator (row
// stride ld) by power iteration on the device
abc_status power_bound(rocblas_handle hnd, DevBufs& db, const double2* mat, int m, int ld, double* bound,
                       std::string& err) {
  std::vector<double2> v0(m);
  for (int i = 0; i < m; ++i) v0[i] = make_double2(std::cos(0.7 * i + 0.1), std::sin(1.3 * i));
  double2 *v = nullptr, *u = nullptr;
  abc_status st = upload(db, &v, v0, err);
  if (st != ABC_OK) return st;
  if (!db.alloc(&u, (size_t)m)) { err = "hipMalloc failed"; return ABC_ENOMEM; }
  const zc one(1.0, 0.0), zero(0.0, 0.0);
  // the growth per iteration is averaged geometrically over the second half
  // of the iterations: for a dominant complex pair the one-step ratio
  // oscillates around the spectral radius, its geometric mean does not
  constexpr int kIters = 120;
  double est = 0, nv = 0, logsum = 0;
  int nlog = 0;
  if (rocblas_dznrm2_64(hnd, m, reinterpret_cast<zc*>(v), 1, &nv) != rocblas_status_success) {
    err = "rocBLAS failed";
    return ABC_EDEVICE;
  }
  for (int it = 0; it < kIters; ++it) {
    // the row-major block is the transpose of a column-major view with lda = ld
    double nu = 0;
    if (rocblas_zgemv_64(hnd, rocblas_operation_transpose, m, m, &one, reinterpret_cast<const zc*>(mat), ld,
                         reinterpret_cast<const zc*>(v), 1, &zero, reinterpret_cast<zc*>(u), 1) !=
            rocblas_status_success ||
        rocblas_dznrm2_64(hnd, m, reinterpret_cast<zc*>(u), 1, &nu) != rocblas_status_success) {
      err = "rocBLAS failed";
      return ABC_EDEVICE;
    }
    if (!(nu > 0)) {
      est = 0;
      nlog = 0;
      break;
    }
    if (it >= kIters / 2) {
      logsum += std::log(nu / nv);
      ++nlog;
    }
    const double sc = 1.0 / nu;
    if (rocblas_zdscal_64(hnd, m, &sc, reinterpret_cast<zc*>(u), 1) != rocblas_status_success) {
      err = "rocBLAS failed";
      return ABC_EDEVICE;
    }
    std::swap(u, v);
    nv = 1.0;
  }
  if (nlog > 0) est = std::exp(logsum / nlog);
  *bound = 1.25 * est;
  return ABC_OK;
}

// [[0, I, A1], [B0, B1, C]] (row-major, ld 3n) from the transposed
// coefficient blocks Y_k = XT + k n (column-major n x n, ld m; k = B1, B0,
// A1, A0), with C = B1 A1 + A0
abc_status assemble_second(rocblas_handle hnd, DevBufs& db, double2* out, const double2* XT, long long m, int n,
                           std::string& err) {
  const double2 one2 = make_double2(1.0, 0.0);
  const zc one(1.0, 0.0);
  double2* W = nullptr;
  if (!db.alloc(&W, (size_t)n * n)) { err = "hipMalloc failed"; return ABC_ENOMEM; }
  // C^T = A1^T B1^T + A0^T: W (column-major, = Y_3 = A0^T) += Y_2 Y_0
  copy2d(W, n, XT + 3LL * n, m, n, n, one2, 0.0);  // row a of W = column a of Y_3: W = Y_3 column-major
  abc_status st = launch_ok(err);
  if (st == ABC_OK &&
      rocblas_zgemm_64(hnd, rocblas_operation_none, rocblas_operation_none, n, n, n, &one,
                       reinterpret_cast<const zc*>(XT + 2LL * n), m, reinterpret_cast<const zc*>(XT), m, &one,
                       reinterpret_cast<zc*>(W), n) != rocblas_status_success) {
    err = "device GEMM for B1 A1 + A0 failed";
    st = ABC_EDEVICE;
  }
  if (st == ABC_OK) {
    // coefficient k at (i, j) is XT[i * m + k n + j]: row i of coefficient
    // k is contiguous; W is C^T column-major, so C(i, j) = W[i * n + j]
    const long long ld = 3LL * n;
    if (hipMemset(out, 0, (size_t)2 * n * ld * 16) != hipSuccess) { err = "hipMemset failed"; st = ABC_EDEVICE; }
    copy2d(out + n, ld, out + n, ld, n, n, make_double2(0.0, 0.0), 1.0);  // identity block
    copy2d(out + 2LL * n, ld, XT + 2LL * n, m, n, n, one2, 0.0);          // A1
    copy2d(out + n * ld, ld, XT + 1LL * n, m, n, n, one2, 0.0);           // B0
    copy2d(out + n * ld + n, ld, XT, m, n, n, one2, 0.0);                 // B1
    copy2d(out + n * ld + 2LL * n, ld, W, n, n, n, one2, 0.0);            // C
    if (st == ABC_OK) st = launch_ok(err);
  }
  db.release(W);
  return st;
}

}  // namespace

abc_status build_box_ops(const abc_params& p, double2** mat_dev, double2** q_dev, int* n_gamma,
                         std::vector<int>& gamma_lin, double* spectral_bound, int* subspace_dim, BoxReduced* reduced,
                         std::string& err) {
  *mat_dev = nullptr;
  *q_dev = nullptr;
  BoxGeom bg = box_geometry(p);
  const int n = (int)bg.glin.size();
  *n_gamma = n;
  if (subspace_dim) *subspace_dim = n;
  gamma_lin = bg.glin;
  const double nn = (double)n * n * 16;
  const double need = p.order == ABC_SECOND ? 36 * nn : (p.order == ABC_FIRST ? 7 * nn : 3 * nn);
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) { err = "hipMemGetInfo failed"; return ABC_EDEVICE; }
  if (need > 0.9 * (double)free_b) {
    err = "box form too large for this box and device (about " + std::to_string((long long)(need / 1e9)) +
          " GB of setup buffers); use the face form";
    return ABC_ENOMEM;
  }
  rocblas_handle hnd;
  if (rocblas_create_handle(&hnd) != rocblas_status_success) { err = "rocblas_create_handle failed"; return ABC_EDEVICE; }
  abc_status st = ABC_OK;
  DevBufs db;
  GammaDev gd;
  gd.n = n;
  if ((st = upload(db, &gd.cnt, bg.cnt, err)) == ABC_OK && (st = upload(db, &gd.cq, bg.cq, err)) == ABC_OK &&
      (st = upload(db, &gd.cw, bg.cw, err)) == ABC_OK)
    st = upload(db, &gd.pos, bg.pos, err);
  const int rows = box_rows(p.order, n), cols = box_cols(p.order, n);
  double2* out = nullptr;  // row-major operator, kept by the context
  double2* Q = nullptr;    // first order: (H_gs H_sg)^{-1}, kept by the context
  if (st == ABC_OK && !db.alloc(&out, (size_t)rows * cols)) { err = "hipMalloc of box operator failed"; st = ABC_ENOMEM; }
  const double2 one2 = make_double2(1.0, 0.0);
  if (st == ABC_OK && p.order == ABC_ZEROTH) {
    double2* K = nullptr;
    st = dtn_matrix(p, gd, p.s0, hnd, db, &K, err);
    if (st == ABC_OK) {
      to_row_major(out, n, K, n, n, n, one2, 0.0);
      st = launch_ok(err);
    }
  } else if (st == ABC_OK && p.order == ABC_FIRST) {
    double2* K1 = nullptr;
    st = dtn_matrix(p, gd, p.s1, hnd, db, &K1, err);
    std::vector<int> hij;
    std::vector<double2> hval;
    gamma_sigma_product(bg, hij, hval);
    int* dij = nullptr;
    double2* dval = nullptr;
    if (st == ABC_OK && (st = upload(db, &dij, hij, err)) == ABC_OK) st = upload(db, &dval, hval, err);
    double2 *HH = nullptr, *Acm = nullptr;
    const size_t nsq = (size_t)n * n;
    if (st == ABC_OK && (!db.alloc(&HH, nsq) || !db.alloc(&Acm, nsq))) { err = "hipMalloc failed"; st = ABC_ENOMEM; }
    if (st == ABC_OK) {
      if (hipMemset(HH, 0, nsq * 16) != hipSuccess) { err = "hipMemset failed"; st = ABC_EDEVICE; }
      scatter_kernel<<<nblk((long long)hval.size()), kThreads>>>(HH, n, dij, dval, (int)hval.size());
      if (st == ABC_OK) st = launch_ok(err);
    }
    if (st == ABC_OK && !(p.s2 > 0)) {
      // theorem pair: A = -i HH, B = s1 I - A K1^{-1} = s1 I - (K1^{-1} A)^T
      // (A and K1 complex symmetric)
      copy2d(Acm, n, HH, n, n, n, make_double2(0.0, -1.0), 0.0);
      double2* X = nullptr;
      if (!db.alloc(&X, nsq)) { err = "hipMalloc failed"; st = ABC_ENOMEM; }
      if (st == ABC_OK && hipMemcpy(X, Acm, nsq * 16, hipMemcpyDeviceToDevice) != hipSuccess) {
        err = "hipMemcpy failed";
        st = ABC_EDEVICE;
      }
      if (st == ABC_OK) st = lu_solve(hnd, db, n, n, K1, X, err, "K(s1)");
      // B(r, c) = s1 delta_rc - X(c, r) = s1 delta_rc - X[r * n + c]
      if (st == ABC_OK) {
        copy2d(out, 2LL * n, X, n, n, n, make_double2(-1.0, 0.0), p.s1);
        st = launch_ok(err);
      }
      db.release(X);
      db.release(K1);
    } else if (st == ABC_OK) {
      // two-point interpolation: (K2 - K1) B^T = s2 K2 - s1 K1, A = s1 K1 - B K1
      double2 *K2 = nullptr, *D = nullptr;
      st = dtn_matrix(p, gd, p.s2, hnd, db, &K2, err);
      if (st == ABC_OK && !db.alloc(&D, nsq)) { err = "hipMalloc failed"; st = ABC_ENOMEM; }
      if (st == ABC_OK) {
        axpby_kernel<<<nblk((long long)nsq), kThreads>>>(D, K2, K1, 1.0, -1.0, (long long)nsq);
        axpby_kernel<<<nblk((long long)nsq), kThreads>>>(K2, K2, K1, p.s2, -p.s1, (long long)nsq);
        st = launch_ok(err);
      }
      if (st == ABC_OK) st = lu_solve(hnd, db, n, n, D, K2, err, "K(s2) - K(s1)");  // K2 <- B^T
      if (st == ABC_OK) {
        // B(r, c) = B^T(c, r) = BT[r * n + c]
        copy2d(out, 2LL * n, K2, n, n, n, one2, 0.0);
        st = launch_ok(err);
      }
      if (st == ABC_OK && hipMemcpy(Acm, K1, nsq * 16, hipMemcpyDeviceToDevice) != hipSuccess) {
        err = "hipMemcpy failed";
        st = ABC_EDEVICE;
      }
      if (st == ABC_OK) {
        const zc alpha(-1.0, 0.0), beta(p.s1, 0.0);
        if (rocblas_zgemm_64(hnd, rocblas_operation_transpose, rocblas_operation_none, n, n, n, &alpha,
                          reinterpret_cast<const zc*>(K2), n, reinterpret_cast<const zc*>(K1), n, &beta,
                          reinterpret_cast<zc*>(Acm), n) != rocblas_status_success) {
          err = "device GEMM for A failed";
          st = ABC_EDEVICE;
        }
      }
      db.release(D);
      db.release(K2);
      db.release(K1);
    }
    if (st == ABC_OK) {
      to_row_major(out + n, 2LL * n, Acm, n, n, n, one2, 0.0);
      st = launch_ok(err);
    }
    db.release(Acm);
    // Q = HH^{-1} (Lyapunov weight of the first-order theorem)
    double2* Qcm = nullptr;
    if (st == ABC_OK && (!db.alloc(&Qcm, nsq) || !db.alloc(&Q, nsq))) { err = "hipMalloc failed"; st = ABC_ENOMEM; }
    if (st == ABC_OK) {
      if (hipMemset(Qcm, 0, nsq * 16) != hipSuccess) { err = "hipMemset failed"; st = ABC_EDEVICE; }
      copy2d(Qcm, n, Qcm, n, n, n, make_double2(0.0, 0.0), 1.0);  // identity
      if (st == ABC_OK) st = launch_ok(err);
    }
    if (st == ABC_OK) st = lu_solve(hnd, db, n, n, HH, Qcm, err, "H_gs H_sg");
    if (st == ABC_OK) {
      to_row_major(Q, n, Qcm, n, n, n, one2, 0.0);
      st = launch_ok(err);
    }
    db.release(Qcm);
    db.release(HH);
  } else if (st == ABC_OK && p.order == ABC_SECOND) {
    // Sec. 3.3: [B1 B0 A1 A0] from one 4r x 4r solve of the transposed
    // interpolation system, r the dimension of the maps' dominant subspace
    // (r = n unless directions fall below kSecondTau; then the reduced maps
    // U^T K_j U are interpolated and each coefficient lifted as U X U^T).
    // X^T(k r + b, a) = coefficient k at (a, b), k = B1, B0, A1, A0
    const double sp[4] = {p.s1, p.s2, p.s3, p.s4};
    FourK fk{};
    double2* Kd[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int j = 0; j < 4 && st == ABC_OK; ++j) st = dtn_matrix(p, gd, sp[j], hnd, db, &Kd[j], err);
    double2* U = nullptr;
    double* Ur = nullptr;
    int r = n;
    if (st == ABC_OK) st = dominant_subspace(hnd, db, n, Kd, &U, &Ur, &r, err);
    const zc one(1.0, 0.0), zero(0.0, 0.0);
    if (st == ABC_OK && U) {
      // K_j <- U^T K_j U (r x r); U is real, so U^T is its adjoint
      double2* T = nullptr;
      if (!db.alloc(&T, (size_t)n * r)) { err = "hipMalloc failed"; st = ABC_ENOMEM; }
      for (int j = 0; j < 4 && st == ABC_OK; ++j) {
        double2* Kr = nullptr;
        if (!db.alloc(&Kr, (size_t)r * r)) { err = "hipMalloc failed"; st = ABC_ENOMEM; break; }
        if (rocblas_zgemm_64(hnd, rocblas_operation_none, rocblas_operation_none, n, r, n, &one,
                             reinterpret_cast<const zc*>(Kd[j]), n, reinterpret_cast<const zc*>(U), n, &zero,
                             reinterpret_cast<zc*>(T), n) != rocblas_status_success ||
            rocblas_zgemm_64(hnd, rocblas_operation_transpose, rocblas_operation_none, r, r, n, &one,
                             reinterpret_cast<const zc*>(U), n, reinterpret_cast<const zc*>(T), n, &zero,
                             reinterpret_cast<zc*>(Kr), r) != rocblas_status_success) {
          err = "device GEMM for the reduced maps failed";
          st = ABC_EDEVICE;
        }
        db.release(Kd[j]);
        Kd[j] = Kr;
      }
      db.release(T);
    }
    const long long m = 4LL * r, mf = 4LL * n;
    double2 *MT = nullptr, *XR = nullptr, *XT = nullptr;
    if (st == ABC_OK && (!db.alloc(&MT, (size_t)(m * m)) || !db.alloc(&XR, (size_t)(m * r)))) {
      err = "hipMalloc failed";
      st = ABC_ENOMEM;
    }
    if (st == ABC_OK) {
      for (int j = 0; j < 4; ++j) { fk.K[j] = Kd[j]; fk.s[j] = sp[j]; }
      dim3 grid(nblk(m), (unsigned)std::min<long long>(m + r, 65535));
      second_system_kernel<<<grid, kThreads>>>(MT, XR, r, fk);
      st = launch_ok(err);
    }
    for (int j = 0; j < 4; ++j) db.release(Kd[j]);
    if (st == ABC_OK) st = lu_solve(hnd, db, (int)m, r, MT, XR, err, "second-order interpolation system");
    db.release(MT);
    // the reduced operator and the basis, for stepping one orbital in the
    // subspace (the lifted operator below serves the orbital batches and
    // the export)
    double2* red = nullptr;
    if (st == ABC_OK && U && reduced) {
      if (!db.alloc(&red, (size_t)2 * r * 3 * r)) { err = "hipMalloc failed"; st = ABC_ENOMEM; }
      if (st == ABC_OK) st = assemble_second(hnd, db, red, XR, m, r, err);
    }
    if (st == ABC_OK && U) {
      // coefficient_k^T = U Y~_k U^T into the full 4n x n layout (ld 4n)
      double2* T = nullptr;
      if (!db.alloc(&XT, (size_t)(mf * n)) || !db.alloc(&T, (size_t)n * r)) { err = "hipMalloc failed"; st = ABC_ENOMEM; }
      for (int k = 0; k < 4 && st == ABC_OK; ++k)
        if (rocblas_zgemm_64(hnd, rocblas_operation_none, rocblas_operation_none, n, r, r, &one,
                             reinterpret_cast<const zc*>(U), n, reinterpret_cast<const zc*>(XR + (long long)k * r), m,
                             &zero, reinterpret_cast<zc*>(T), n) != rocblas_status_success ||
            rocblas_zgemm_64(hnd, rocblas_operation_none, rocblas_operation_transpose, n, n, r, &one,
                             reinterpret_cast<const zc*>(T), n, reinterpret_cast<const zc*>(U), n, &zero,
                             reinterpret_cast<zc*>(XT + (long long)k * n), mf) != rocblas_status_success) {
          err = "device GEMM lifting the second-order coefficients failed";
          st = ABC_EDEVICE;
        }
      db.release(T);
      db.release(XR);
      db.release(U);
    } else {
      XT = XR;
    }
    if (st == ABC_OK) st = assemble_second(hnd, db, out, XT, mf, n, err);
    db.release(XT);
    if (subspace_dim) *subspace_dim = r;
    if (st == ABC_OK && red && reduced) {
      // the stepping reads U by columns (projection) and by rows (lift)
      double* Ut = nullptr;
      if (!db.alloc(&Ut, (size_t)n * r)) {
        err = "hipMalloc failed";
        st = ABC_ENOMEM;
      } else {
        transpose_real_kernel<<<nblk((long long)n * r), kThreads>>>(Ut, Ur, n, r);
        if (hipGetLastError() != hipSuccess) { err = "setup kernel launch failed"; st = ABC_EDEVICE; }
      }
      if (st == ABC_OK) {
        reduced->U = Ur;
        reduced->Ut = Ut;
        reduced->red = red;
        reduced->r = r;
      }
    }
  }
  // spectral radius of M (zeroth), B (first) or the (f, g) block
  // [[0, I], [B0, B1]] (second), with a safety factor; the row-sum norm of
  // these dense non-normal matrices is far above their spectral radius
  double bound = 0;
  if (st == ABC_OK) st = power_bound(hnd, db, out, p.order == ABC_ZEROTH ? n : box_aux_rows(p.order, n), cols,
                                     &bound, err);
  if (st == ABC_OK && hipDeviceSynchronize() != hipSuccess) { err = "box-form setup failed on the device"; st = ABC_EDEVICE; }
  rocblas_destroy_handle(hnd);
  if (st != ABC_OK) {
    if (reduced) *reduced = BoxReduced{};  // freed with the other setup buffers
    return st;
  }
  *spectral_bound = bound;
  db.keep(out);
  *mat_dev = out;
  if (reduced && reduced->red) {
    db.keep(reduced->red);
    db.keep(reduced->U);
    db.keep(reduced->Ut);
  }
  if (Q) {
    db.keep(Q);
    *q_dev = Q;
  }
  return ABC_OK;
}

}  // namespace abc
