// Stage-by-stage kernels for the Taylor-4 step with the DtN boundary
// conditions.  One launch per stage for the box sweep plus one per stage for
// the boundary operator; this path handles every order, form, kernel width
// and precision and is the reference the fused kernel is checked against.
//
// A stage computes z_k = (dt/k) L z_{k-1} for the generator
//   L(psi, f) = (-i H psi - i E^T f,  B f + A E psi)        (first order)
//   L psi     = -i (H psi + E^T M E psi)                   (zeroth order)
//   L(psi, f, g) = (-i H psi - i E^T f,  g + A1 E psi,
//                   B1 g + B0 f + (B1 A1 + A0) E psi)      (second order)
// (Sec. 3 dynamics) and accumulates z_0 + ... + z_4 (Sec. 4 Taylor step).
// The second order exists in the box form only; its boundary variables
// [f; g] are one vector of 2 n_Gamma rows for the box operator.
#include <hip/hip_runtime.h>

#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>

#include "abc_internal.h"

using abc::Geometry;

namespace {

template <typename T> struct cpx;
template <> struct cpx<double> { using t = double2; };
template <> struct cpx<float> { using t = float2; };

constexpr int kBlock = 256;

struct StencilCoef {
  double diag;               // -(3 c_0) / (2 h^2)
  double off[abc::kMaxR + 1];  // -c_k / (2 h^2), k >= 1
};

__device__ __forceinline__ long long lin(const Geometry& g, int x, int y, int z) {
  return ((long long)z * g.ny + y) * g.nx + x;
}

// linear index of face element (f, layer, t1, t2) in the box
__device__ __forceinline__ long long face_point(const Geometry& g, int f, int l, int t1, int t2) {
  switch (f) {
    case 0: return lin(g, l, t2, t1);
    case 1: return lin(g, g.nx - 1 - l, t2, t1);
    case 2: return lin(g, t2, l, t1);
    case 3: return lin(g, t2, g.ny - 1 - l, t1);
    case 4: return lin(g, t2, t1, l);
    default: return lin(g, t2, t1, g.nz - 1 - l);
  }
}

// sum over the faces containing point (x, y, z) of the face buffer value
__device__ __forceinline__ double2 face_gather(const Geometry& g, const double2* __restrict__ fb,
                                               int x, int y, int z, int b) {
  double2 s = make_double2(0.0, 0.0);
  const int R = g.R, B = g.batch;
  auto add = [&](int f, int l, int t1, int t2) {
    const double2 v = fb[g.face_off[f] + (((long long)l * g.face_n1[f] + t1) * g.face_n2[f] + t2) * B + b];
    s.x += v.x;
    s.y += v.y;
  };
  if (x < R) add(0, x, z, y);
  if (x >= g.nx - R) add(1, g.nx - 1 - x, z, y);
  if (y < R) add(2, y, z, x);
  if (y >= g.ny - R) add(3, g.ny - 1 - y, z, x);
  if (z < R) add(4, z, y, x);
  if (z >= g.nz - R) add(5, g.nz - 1 - z, y, x);
  return s;
}

// ---------------------------------------------------------------------------
// mean field: veff = V + t0 rho + t3 rho^2, rho = sum_b |psi_b|^2
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) meanfield_kernel(const typename cpx<T>::t* __restrict__ psi,
                                                           const T* __restrict__ V, T* __restrict__ veff,
                                                           long long npts, int batch, T t0, T t3) {
  long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  T rho = 0;
  for (int b = 0; b < batch; ++b) {
    auto v = psi[p * batch + b];
    rho += v.x * v.x + v.y * v.y;
  }
  T base = V ? V[p] : T(0);
  veff[p] = base + t0 * rho + t3 * rho * rho;
}

// ---------------------------------------------------------------------------
// box sweep of one stage
// The running Taylor sum psi + z_1 + z_2 + z_3 + z_4 is formed by stages 2
// and 4 from their own input (z_1, z_3) and the sum so far, in the order of
// a running sum, so stages 1 and 3 only write their z:
// mode 0: y_out = y_new                                (stages 1, 3)
// mode 1: acc = (state + y_in) + y_new, y_out = y_new  (stage 2; state = psi)
// mode 2: state = (acc + y_in) + y_new                 (stage 4: the new psi)
// The face kernels keep their own modes 0 (stage 1), 1 (stages 2, 3) and 2.
// ---------------------------------------------------------------------------
// the rest of a stage at point p (orbital b, element e) once the stencil sum
// (hr, hi) is formed: potential, boundary source, -i coef, and the mode's
// accumulator update
// (vv = V[p] when V is given, av = state[e] in mode 1 and acc[e] in mode 2:
// loaded by the caller, so that a sweep can issue them early)
template <typename T, int R>
__device__ __forceinline__ void stage_tail(long long e, long long p, int b, int x, int y, int z,
                                           const typename cpx<T>::t c0, T hr, T hi, T vv, typename cpx<T>::t av,
                                           typename cpx<T>::t* __restrict__ acc, typename cpx<T>::t* __restrict__ yout,
                                           typename cpx<T>::t* __restrict__ state, const T* __restrict__ V,
                                           const double2* __restrict__ fsrc, const double2* __restrict__ bsrc,
                                           const int* __restrict__ point_gamma, const Geometry& g, double coef,
                                           int mode) {
  using C = typename cpx<T>::t;
  if (V) {
    hr += vv * c0.x;
    hi += vv * c0.y;
  }
  // boundary term (FP64 source, added in the stencil precision)
  if (fsrc) {
    if (x < R || x >= g.nx - R || y < R || y >= g.ny - R || z < R || z >= g.nz - R) {
      const double2 s = face_gather(g, fsrc, x, y, z, b);
      hr += T(s.x);
      hi += T(s.y);
    }
  } else if (bsrc) {
    const int gi = point_gamma[p];
    if (gi >= 0) {
      const double2 s = bsrc[(long long)gi * g.batch + b];
      hr += T(s.x);
      hi += T(s.y);
    }
  }
  // y_new = coef * (-i) (H y + src)
  const T cf = T(coef);
  C yn;
  yn.x = cf * hi;
  yn.y = -cf * hr;
  C a;
  a.x = (av.x + c0.x) + yn.x;
  a.y = (av.y + c0.y) + yn.y;
  if (mode == 0) {
    yout[e] = yn;
  } else if (mode == 1) {
    acc[e] = a;
    yout[e] = yn;
  } else {
    state[e] = a;
  }
}

template <typename T, int R, bool PER>
__device__ __forceinline__ void stage_body(
    long long e, const typename cpx<T>::t* __restrict__ yin, typename cpx<T>::t* __restrict__ yout,
    typename cpx<T>::t* __restrict__ acc, typename cpx<T>::t* __restrict__ state,
    const T* __restrict__ V, const double2* __restrict__ fsrc, const double2* __restrict__ bsrc,
    const int* __restrict__ point_gamma, const Geometry& g, const StencilCoef& sc, double coef, int mode) {
  using C = typename cpx<T>::t;
  const int B = g.batch;
  if (e >= g.npts * B) return;
  long long p;
  int b, x, y, z;
  if (g.npts * B <= 0x7fffffffLL) {  // 32-bit index arithmetic (64-bit division is a long software routine)
    const unsigned ue = (unsigned)e, up = ue / (unsigned)B, r = up / (unsigned)g.nx;
    p = up;
    b = (int)(ue - up * (unsigned)B);
    x = (int)(up - r * (unsigned)g.nx);
    z = (int)(r / (unsigned)g.ny);
    y = (int)(r - (unsigned)z * (unsigned)g.ny);
  } else {
    p = e / B;
    b = (int)(e - p * B);
    x = (int)(p % g.nx);
    y = (int)((p / g.nx) % g.ny);
    z = (int)(p / ((long long)g.nx * g.ny));
  }
  const C c0 = yin[e];
  T hr = T(sc.diag) * c0.x, hi = T(sc.diag) * c0.y;
  const long long sx = B, sy = (long long)g.nx * B, sz = (long long)g.nx * g.ny * B;
#pragma unroll
  for (int k = 1; k <= R; ++k) {
    const T w = T(sc.off[k]);
    T ar = 0, ai = 0;
    if (PER) {
      const int xp = (x + k) % g.nx, xm = (x - k + g.nx) % g.nx;
      const int yp = (y + k) % g.ny, ym = (y - k + g.ny) % g.ny;
      const int zp = (z + k) % g.nz, zm = (z - k + g.nz) % g.nz;
      const C v0 = yin[(lin(g, xp, y, z)) * B + b], v1 = yin[(lin(g, xm, y, z)) * B + b];
      const C v2 = yin[(lin(g, x, yp, z)) * B + b], v3 = yin[(lin(g, x, ym, z)) * B + b];
      const C v4 = yin[(lin(g, x, y, zp)) * B + b], v5 = yin[(lin(g, x, y, zm)) * B + b];
      ar = v0.x + v1.x + v2.x + v3.x + v4.x + v5.x;
      ai = v0.y + v1.y + v2.y + v3.y + v4.y + v5.y;
    } else {
      if (x + k < g.nx) { C v = yin[e + k * sx]; ar += v.x; ai += v.y; }
      if (x - k >= 0) { C v = yin[e - k * sx]; ar += v.x; ai += v.y; }
      if (y + k < g.ny) { C v = yin[e + k * sy]; ar += v.x; ai += v.y; }
      if (y - k >= 0) { C v = yin[e - k * sy]; ar += v.x; ai += v.y; }
      if (z + k < g.nz) { C v = yin[e + k * sz]; ar += v.x; ai += v.y; }
      if (z - k >= 0) { C v = yin[e - k * sz]; ar += v.x; ai += v.y; }
    }
    hr += w * ar;
    hi += w * ai;
  }
  C av;
  av.x = 0;
  av.y = 0;
  if (mode == 1) av = state[e];
  else if (mode == 2) av = acc[e];
  stage_tail<T, R>(e, p, b, x, y, z, c0, hr, hi, V ? V[p] : T(0), av, acc, yout, state, V, fsrc, bsrc, point_gamma,
                   g, coef, mode);
}

template <typename T, int R, bool PER>
__global__ void __launch_bounds__(kBlock) stage_kernel(
    const typename cpx<T>::t* __restrict__ yin, typename cpx<T>::t* __restrict__ yout,
    typename cpx<T>::t* __restrict__ acc, typename cpx<T>::t* __restrict__ state,
    const T* __restrict__ V, const double2* __restrict__ fsrc, const double2* __restrict__ bsrc,
    const int* __restrict__ point_gamma, Geometry g, StencilCoef sc, double coef, int mode) {
  stage_body<T, R, PER>((long long)blockIdx.x * blockDim.x + threadIdx.x, yin, yout, acc, state, V, fsrc, bsrc,
                        point_gamma, g, sc, coef, mode);
}

// ---------------------------------------------------------------------------
// the same sweep tiled, for one orbital with zero outside the box: a
// workgroup owns kTX x-columns, TY = TW J rows (wave w takes rows w, w + TW,
// ...) and tz planes, and marches z.  Each thread keeps its J points' 2R + 1
// z-neighbours in a register queue that advances one plane per step, so the
// tile's interior is read from memory once; the centre plane goes to LDS with
// R-wide x and y halos (double buffered: one barrier per plane) for the x
// and y neighbours.  The next plane's loads are issued before the barrier.
// ---------------------------------------------------------------------------
constexpr int kTX = 64;
// one row per thread; planes per tile and rows per tile by radius (measured
// at 128^3, us per step, first order w = 0: with 4 rows, R = 3 136 with 16
// planes against 142 with 8 and 193 with 32, R = 2 117 with 8 against 122
// with 16, two rows per thread 143 and 129; R = 1, w = 8: 136 with 8 planes,
// 157 with 16, 159 untiled.  Same-box A/B of the row count: R = 3 129.7 with
// 4 rows x 16 planes, 129.5 with 8 x 16, 122.9 with 8 x 8, 127.9 with 16 x 8;
// R = 2 106.0 with 4 x 8, 101.5 with 8 x 8: the y halo's share of each
// plane's loads halves at 8 rows).
constexpr int kTileJ = 1;
constexpr int kTiledMinR = 1;
constexpr int tile_planes(int R) { return 8; }
// threads per tile (one row each): kTiledBlock(R) / 64 rows
constexpr int kTiledBlock(int R) { return R >= 2 ? 512 : 256; }

struct TileGrid {
  int ntx, nty, ntz, tz;
  int tiles_per_xcd;  // tiles / 8 when that divides, for the XCD-aware order; else 0
};

template <int R, int J>
struct TileShape {
  static constexpr int NTB = kTiledBlock(R), TW = NTB / 64;  // threads, waves (rows per pass)
  static constexpr int TY = TW * J, LX = kTX + 2 * R, LY = TY + 2 * R;
  static constexpr int NH = 2 * R * (kTX + TY);        // halo points per plane
  static constexpr int HPT = (NH + NTB - 1) / NTB;     // per thread
};

template <typename T, int R, int J>
__device__ __forceinline__ void stage_tiled_body(
    int tile, const TileGrid& tg, const typename cpx<T>::t* __restrict__ yin, typename cpx<T>::t* __restrict__ yout,
    typename cpx<T>::t* __restrict__ acc, typename cpx<T>::t* __restrict__ state, const T* __restrict__ V,
    const double2* __restrict__ fsrc, const double2* __restrict__ bsrc, const int* __restrict__ point_gamma,
    const Geometry& g, const StencilCoef& sc, double coef, int mode) {
  using C = typename cpx<T>::t;
  using S = TileShape<R, J>;
  __shared__ C pl[2][S::LY][S::LX];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int bx = tile % tg.ntx, by = (tile / tg.ntx) % tg.nty, bz = tile / (tg.ntx * tg.nty);
  const int x0 = bx * kTX, y0 = by * S::TY, z0 = bz * tg.tz;
  const int z1 = min(z0 + tg.tz, g.nz);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const long long sy = nx, sz = (long long)nx * ny;
  const int x = x0 + tx;
  auto load = [&](int xx, int yy, int zz) {
    C v;
    v.x = 0;
    v.y = 0;
    if (xx >= 0 && xx < nx && yy >= 0 && yy < ny && zz >= 0 && zz < nz) v = yin[zz * sz + yy * sy + xx];
    return v;
  };
  // halo point h of a plane: LDS position and box coordinates
  auto halo_pos = [&](int h, int& ly, int& lx) {
    if (h < 2 * R * kTX) {
      const int r = h / kTX, c = h % kTX;
      ly = r < R ? r : S::TY + r;
      lx = R + c;
    } else {
      const int k = h - 2 * R * kTX, r = k % S::TY, c = k / S::TY;
      ly = R + r;
      lx = c < R ? c : kTX + c;
    }
  };
  C q[J][2 * R + 1];
  C hv[S::HPT];
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int i = 0; i <= 2 * R; ++i) q[j][i] = load(x, y0 + ty + S::TW * j, z0 - R + i);
#pragma unroll
  for (int hh = 0; hh < S::HPT; ++hh) {
    const int h = threadIdx.x + hh * S::NTB;
    int ly = 0, lx = 0;
    if (h < S::NH) halo_pos(h, ly, lx);
    hv[hh] = load(x0 - R + lx, y0 - R + ly, h < S::NH ? z0 : -1);
  }
  const T diag = T(sc.diag);
  T off[R + 1];
#pragma unroll
  for (int k = 1; k <= R; ++k) off[k] = T(sc.off[k]);
  for (int z = z0; z < z1; ++z) {
    const int buf = (z - z0) & 1;
#pragma unroll
    for (int j = 0; j < J; ++j) pl[buf][R + ty + S::TW * j][R + tx] = q[j][R];
#pragma unroll
    for (int hh = 0; hh < S::HPT; ++hh) {
      const int h = threadIdx.x + hh * S::NTB;
      if (h < S::NH) {
        int ly, lx;
        halo_pos(h, ly, lx);
        pl[buf][ly][lx] = hv[hh];
      }
    }
    T vv[J];
    C av[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int yy = y0 + ty + S::TW * j;
      const long long pnt = z * sz + yy * sy + x;
      const bool in = x < nx && yy < ny;
      vv[j] = (V && in) ? V[pnt] : T(0);
      av[j].x = 0;
      av[j].y = 0;
      if (mode != 0 && in) av[j] = mode == 1 ? state[pnt] : acc[pnt];
    }
    C nxt[J];
    const bool more = z + 1 < z1;
#pragma unroll
    for (int j = 0; j < J; ++j) nxt[j] = load(x, y0 + ty + S::TW * j, more ? z + R + 1 : -1);
#pragma unroll
    for (int hh = 0; hh < S::HPT; ++hh) {
      const int h = threadIdx.x + hh * S::NTB;
      int ly = 0, lx = 0;
      if (h < S::NH) halo_pos(h, ly, lx);
      hv[hh] = load(x0 - R + lx, y0 - R + ly, (more && h < S::NH) ? z + 1 : -1);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int yy = y0 + ty + S::TW * j, ly = R + ty + S::TW * j, lx = R + tx;
      const C c0 = q[j][R];
      T hr = diag * c0.x, hi = diag * c0.y;
#pragma unroll
      for (int k = 1; k <= R; ++k) {
        const C a0 = pl[buf][ly][lx + k], a1 = pl[buf][ly][lx - k];
        const C a2 = pl[buf][ly + k][lx], a3 = pl[buf][ly - k][lx];
        const C a4 = q[j][R + k], a5 = q[j][R - k];
        hr += off[k] * (((a0.x + a1.x) + (a2.x + a3.x)) + (a4.x + a5.x));
        hi += off[k] * (((a0.y + a1.y) + (a2.y + a3.y)) + (a4.y + a5.y));
      }
      if (x < nx && yy < ny) {
        const long long pnt = z * sz + yy * sy + x;
        stage_tail<T, R>(pnt, pnt, 0, x, yy, z, c0, hr, hi, vv[j], av[j], acc, yout, state, V, fsrc, bsrc,
                         point_gamma, g, coef, mode);
      }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
#pragma unroll
      for (int i = 0; i < 2 * R; ++i) q[j][i] = q[j][i + 1];
      q[j][2 * R] = nxt[j];
    }
  }
}

inline TileGrid make_tile_grid(const Geometry& g, int TY, int tz) {
  TileGrid tg;
  tg.ntx = (g.nx + kTX - 1) / kTX;
  tg.nty = (g.ny + TY - 1) / TY;
  tg.tz = tz;
  tg.ntz = (g.nz + tz - 1) / tz;
  const int n = tg.ntx * tg.nty * tg.ntz;
  tg.tiles_per_xcd = n % 8 == 0 ? n / 8 : 0;
  return tg;
}

__device__ __forceinline__ int xcd_tile(int bid, const TileGrid& tg) {
  return tg.tiles_per_xcd ? (bid & 7) * tg.tiles_per_xcd + (bid >> 3) : bid;
}

template <typename T, int R, int J>
__global__ void __launch_bounds__(kTiledBlock(R)) stage_tiled_kernel(
    TileGrid tg, const typename cpx<T>::t* __restrict__ yin, typename cpx<T>::t* __restrict__ yout,
    typename cpx<T>::t* __restrict__ acc, typename cpx<T>::t* __restrict__ state, const T* __restrict__ V,
    const double2* __restrict__ fsrc, const double2* __restrict__ bsrc, const int* __restrict__ point_gamma,
    Geometry g, StencilCoef sc, double coef, int mode) {
  stage_tiled_body<T, R, J>(xcd_tile(blockIdx.x, tg), tg, yin, yout, acc, state, V, fsrc, bsrc, point_gamma, g,
                            sc, coef, mode);
}

// ---------------------------------------------------------------------------
// face-form boundary operator, one thread per face element (f, l, t1, t2, b)
// first order: g_out = coef (B g_in + A E y);  mode as above for (facc, aux)
// zeroth order: src = M E y
// ---------------------------------------------------------------------------
struct LocalBlock {
  double2 m[abc::kMaxR * abc::kMaxR];
};

template <typename T, int R>
__device__ __forceinline__ void face_body(
    long long e, const double2* __restrict__ gin, double2* __restrict__ gout, double2* __restrict__ facc,
    double2* __restrict__ aux_out, const typename cpx<T>::t* __restrict__ yin,
    const double2* __restrict__ ker, const LocalBlock& a, const Geometry& g, int w, double coef, int mode,
    int first) {
  const int B = g.batch;
  if (e >= g.face_off[6]) return;
  int f = 0;
  while (e >= g.face_off[f + 1]) ++f;
  const long long r = e - g.face_off[f];
  const int n1 = g.face_n1[f], n2 = g.face_n2[f];
  const int b = (int)(r % B);
  const long long q = r / B;
  const int t2 = (int)(q % n2);
  const int t1 = (int)((q / n2) % n1);
  const int l = (int)(q / ((long long)n1 * n2));
  const int K = 2 * w + 1;
  double sr = 0, si = 0;
  const int j1lo = max(0, t1 - w), j1hi = min(n1 - 1, t1 + w);
  const int j2lo = max(0, t2 - w), j2hi = min(n2 - 1, t2 + w);
  for (int lp = 0; lp < R; ++lp) {
    const double2* kl = ker + ((long long)(l * R + lp)) * K * K;
    for (int j1 = j1lo; j1 <= j1hi; ++j1) {
      const double2* krow = kl + (long long)(t1 - j1 + w) * K;
      for (int j2 = j2lo; j2 <= j2hi; ++j2) {
        const double2 kv = krow[t2 - j2 + w];
        double2 v;
        if (first) {
          v = gin[g.face_off[f] + (((long long)lp * n1 + j1) * n2 + j2) * B + b];
        } else {
          const auto yv = yin[face_point(g, f, lp, j1, j2) * B + b];
          v = make_double2((double)yv.x, (double)yv.y);
        }
        sr += kv.x * v.x - kv.y * v.y;
        si += kv.x * v.y + kv.y * v.x;
      }
    }
  }
  if (!first) {
    gout[e] = make_double2(sr, si);
    return;
  }
  for (int lp = 0; lp < R; ++lp) {
    const double2 av = a.m[l * R + lp];
    const auto yv = yin[face_point(g, f, lp, t1, t2) * B + b];
    const double yr = (double)yv.x, yi = (double)yv.y;
    sr += av.x * yr - av.y * yi;
    si += av.x * yi + av.y * yr;
  }
  const double2 gn = make_double2(coef * sr, coef * si);
  if (mode == 0) {
    const double2 g0 = gin[e];
    facc[e] = make_double2(g0.x + gn.x, g0.y + gn.y);
    gout[e] = gn;
  } else if (mode == 1) {
    double2 s = facc[e];
    s.x += gn.x;
    s.y += gn.y;
    facc[e] = s;
    gout[e] = gn;
  } else {
    const double2 s = facc[e];
    aux_out[e] = make_double2(s.x + gn.x, s.y + gn.y);
  }
}

template <typename T, int R>
__global__ void __launch_bounds__(kBlock) face_kernel(
    const double2* __restrict__ gin, double2* __restrict__ gout, double2* __restrict__ facc,
    double2* __restrict__ aux_out, const typename cpx<T>::t* __restrict__ yin,
    const double2* __restrict__ ker, LocalBlock a, Geometry g, int w, double coef, int mode,
    int first) {
  face_body<T, R>((long long)blockIdx.x * blockDim.x + threadIdx.x, gin, gout, facc, aux_out, yin, ker, a, g, w,
                  coef, mode, first);
}

// Face-form boundary operator with a window (w >= 2), one orbital: the same
// sum as face_kernel, tiled.  A workgroup computes a kFT x kFT tile of one
// face layer l.  The input it needs ((kFT + 2w)^2 points of each source
// layer, zero outside the face) and the taps are staged in LDS once; a tap
// read is the same address for the whole wave.  Each output is summed by
// kFSplit threads over interleaved tap rows and combined in LDS: the faces
// are small (6 n^2 outputs), and one thread per output leaves too few waves
// to hide the latency of the multiply-add chains.  The first order's local
// A E y term and the stage update follow as in face_kernel.
constexpr int kFT = 16, kFSplit = 4, kFBlock = kFT * kFT * kFSplit;  // 16 x 16 outputs, 4 threads each
constexpr int kFaceInMax = 3072, kFaceTapMax = 1024;                  // LDS, in double2
inline bool face_tiled_ok(int R, int w, int batch) {
  const int K = 2 * w + 1, S = kFT + 2 * w;
  return batch == 1 && w >= 2 && R * S * S <= kFaceInMax && R * K * K <= kFaceTapMax;
}

template <typename T, int R>
__global__ void __launch_bounds__(kFBlock) face_tiled_kernel(
    const double2* __restrict__ gin, double2* __restrict__ gout, double2* __restrict__ facc,
    double2* __restrict__ aux_out, const typename cpx<T>::t* __restrict__ yin,
    const double2* __restrict__ ker, LocalBlock a, Geometry g, int w, double coef, int mode, int first) {
  __shared__ double2 tin[kFaceInMax];
  __shared__ double2 tap[kFaceTapMax];
  __shared__ double2 part[kFSplit - 1][kFT * kFT];
  const int f = blockIdx.y / R, l = blockIdx.y - f * R;
  const int n1 = g.face_n1[f], n2 = g.face_n2[f];
  const int nt2 = (n2 + kFT - 1) / kFT;
  if ((int)blockIdx.x >= ((n1 + kFT - 1) / kFT) * nt2) return;  // past this face's tiles
  const int t1b = ((int)blockIdx.x / nt2) * kFT, t2b = ((int)blockIdx.x % nt2) * kFT;
  const int S = kFT + 2 * w, K = 2 * w + 1;
  for (int lp = 0; lp < R; ++lp) {
    for (int i = threadIdx.x; i < S * S; i += kFBlock) {
      const int a1 = i / S, a2 = i - a1 * S;
      const int j1 = t1b - w + a1, j2 = t2b - w + a2;
      double2 v = make_double2(0, 0);
      if (j1 >= 0 && j1 < n1 && j2 >= 0 && j2 < n2) {
        if (first) {
          v = gin[g.face_off[f] + ((long long)lp * n1 + j1) * n2 + j2];
        } else {
          const auto yv = yin[face_point(g, f, lp, j1, j2)];
          v = make_double2((double)yv.x, (double)yv.y);
        }
      }
      tin[(lp * S + a1) * S + a2] = v;
    }
    // taps reversed, so that the input and the tap run the same direction
    const double2* kl = ker + (long long)(l * R + lp) * K * K;
    for (int i = threadIdx.x; i < K * K; i += kFBlock) tap[lp * K * K + i] = kl[K * K - 1 - i];
  }
  __syncthreads();
  // thread (q, o): output o of the tile, tap rows d1 = q, q + kFSplit, ...
  const int q = threadIdx.x / (kFT * kFT), o = threadIdx.x - q * (kFT * kFT);
  const int o1 = o / kFT, o2 = o - o1 * kFT;
  double sr = 0, si = 0;
  for (int lp = 0; lp < R; ++lp) {
    for (int d1 = q; d1 < K; d1 += kFSplit) {
      const double2* irow = tin + (lp * S + o1 + d1) * S + o2;
      const double2* krow = tap + lp * K * K + d1 * K;
#pragma unroll 4
      for (int d2 = 0; d2 < K; ++d2) {
        const double2 kv = krow[d2];
        const double2 v = irow[d2];
        sr += kv.x * v.x - kv.y * v.y;
        si += kv.x * v.y + kv.y * v.x;
      }
    }
  }
  if (q > 0) part[q - 1][o] = make_double2(sr, si);
  __syncthreads();
  if (q > 0) return;
#pragma unroll
  for (int p = 0; p < kFSplit - 1; ++p) {
    sr += part[p][o].x;
    si += part[p][o].y;
  }
  const int t1 = t1b + o1, t2 = t2b + o2;
  if (t1 >= n1 || t2 >= n2) return;
  const long long e = g.face_off[f] + ((long long)l * n1 + t1) * n2 + t2;
  if (!first) {
    gout[e] = make_double2(sr, si);
    return;
  }
  for (int lp = 0; lp < R; ++lp) {
    const double2 av = a.m[l * R + lp];
    const auto yv = yin[face_point(g, f, lp, t1, t2)];
    const double yr = (double)yv.x, yi = (double)yv.y;
    sr += av.x * yr - av.y * yi;
    si += av.x * yi + av.y * yr;
  }
  const double2 gn = make_double2(coef * sr, coef * si);
  if (mode == 0) {
    const double2 g0 = gin[e];
    facc[e] = make_double2(g0.x + gn.x, g0.y + gn.y);
    gout[e] = gn;
  } else if (mode == 1) {
    double2 sacc = facc[e];
    sacc.x += gn.x;
    sacc.y += gn.y;
    facc[e] = sacc;
    gout[e] = gn;
  } else {
    const double2 sacc = facc[e];
    aux_out[e] = make_double2(sacc.x + gn.x, sacc.y + gn.y);
  }
}

// A stage and its boundary-variable stage in one launch, for the orders whose
// stage reads the auxiliary input rather than the boundary kernel's output
// (first and second) and a local face operator: the first nsb blocks run the
// stage, the rest the face elements.  It saves a launch and the gap before
// it per stage.
template <typename T, int R, bool PER>
__global__ void __launch_bounds__(kBlock) stage_face_kernel(
    const typename cpx<T>::t* __restrict__ yin, typename cpx<T>::t* __restrict__ yout,
    typename cpx<T>::t* __restrict__ acc, typename cpx<T>::t* __restrict__ state,
    const T* __restrict__ V, const double2* __restrict__ fsrc, const int* __restrict__ point_gamma,
    StencilCoef sc, const double2* __restrict__ gin, double2* __restrict__ gout, double2* __restrict__ facc,
    double2* __restrict__ aux_out, const double2* __restrict__ ker, LocalBlock a, Geometry g, int w, double coef,
    int mode, int fmode, unsigned nsb) {
  if (blockIdx.x < nsb)
    stage_body<T, R, PER>((long long)blockIdx.x * blockDim.x + threadIdx.x, yin, yout, acc, state, V, fsrc, nullptr,
                          point_gamma, g, sc, coef, mode);
  else
    face_body<T, R>((long long)(blockIdx.x - nsb) * blockDim.x + threadIdx.x, gin, gout, facc, aux_out, yin, ker, a,
                    g, w, coef, fmode, 1);
}

// the same with the tiled stage sweep in the first tg tiles
template <typename T, int R, int J>
__global__ void __launch_bounds__(kTiledBlock(R)) stage_face_tiled_kernel(
    TileGrid tg, const typename cpx<T>::t* __restrict__ yin, typename cpx<T>::t* __restrict__ yout,
    typename cpx<T>::t* __restrict__ acc, typename cpx<T>::t* __restrict__ state, const T* __restrict__ V,
    const double2* __restrict__ fsrc, const int* __restrict__ point_gamma, StencilCoef sc,
    const double2* __restrict__ gin, double2* __restrict__ gout, double2* __restrict__ facc,
    double2* __restrict__ aux_out, const double2* __restrict__ ker, LocalBlock a, Geometry g, int w, double coef,
    int mode, int fmode, unsigned nsb) {
  if (blockIdx.x < nsb)
    stage_tiled_body<T, R, J>(xcd_tile(blockIdx.x, tg), tg, yin, yout, acc, state, V, fsrc, nullptr, point_gamma,
                              g, sc, coef, mode);
  else
    face_body<T, R>((long long)(blockIdx.x - nsb) * blockDim.x + threadIdx.x, gin, gout, facc, aux_out, yin, ker, a,
                    g, w, coef, fmode, 1);
}

// ---------------------------------------------------------------------------
// exact face sections by FFT.  Per face pair q (faces 2q, 2q + 1) the slabs
// s = (side R + l) B + b of P1 x P2 points ([t1][t2]) hold the zero-padded
// face layers; the circular convolution with the padded kernel equals the
// Toeplitz section on the n1 x n2 face because P >= 2 n - 1.  A stage takes
// three launches, each over the three face pairs (pair = blockIdx.y):
//   rows:    the face layers, zero-extended along t2, transformed along t2
//            into W (only the n1 rows that hold data: the padded rows are
//            zero and stay zero under a transform along t2);
//   columns: per column of the R layers of one (side, batch) slab group, the
//            forward transform along t1 (rows >= n1 taken as zero), the
//            product with the R x R kernel spectra, and the inverse transform,
//            written to Z for the rows t1 < n1 only;
//   inverse rows + epilogue: the inverse transform along t2 of those rows,
//            then the face_kernel epilogue on t2 < n2.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 twiddle(const double2* tw, int k, bool cj) {
  double2 w = tw[k];
  if (cj) w.y = -w.y;
  return w;
}

// decimation in time: TW lines of L = 2^logL points ([t][k]) held in
// bit-reversed order in buf are transformed in place to natural order; tw[k]
// = exp(+-2 pi i k / L), k < L/2 (cj: its conjugate, the opposite sign; tw
// may sit in LDS or in global memory).  Two radix-2 stages per pass: each
// thread takes four points i + {0, 1, 2, 3} h of a 4h block through stage
// sh (span 2h) and stage sh + 1 (span 4h), so a pass is one LDS round trip
// and one barrier; an odd logL leaves one radix-2 stage.  L, the spans and h
// are powers of two: shifts and masks.  Ends with a barrier.
__device__ __forceinline__ void fft_dit(double2* buf, const double2* tw, int L, int logL, int TW, bool cj = false) {
  int sh = 1;
  for (; sh + 1 <= logL; sh += 2) {
    const int h = 1 << (sh - 1), s1 = L >> sh, s2 = L >> (sh + 1), nq = TW * L / 4;
    for (int q = threadIdx.x; q < nq; q += blockDim.x) {
      const int t = q >> (logL - 2), r = q & ((L >> 2) - 1);
      const int pos = r & (h - 1), i = t * L + ((r >> (sh - 1)) << (sh + 1)) + pos;
      const double2 w1 = twiddle(tw, pos * s1, cj);
      const double2 a = buf[i], b = cmul(buf[i + h], w1), c = buf[i + 2 * h], d = cmul(buf[i + 3 * h], w1);
      const double2 a1 = make_double2(a.x + b.x, a.y + b.y), b1 = make_double2(a.x - b.x, a.y - b.y);
      const double2 c1 = cmul(make_double2(c.x + d.x, c.y + d.y), twiddle(tw, pos * s2, cj));
      const double2 d1 = cmul(make_double2(c.x - d.x, c.y - d.y), twiddle(tw, (pos + h) * s2, cj));
      buf[i] = make_double2(a1.x + c1.x, a1.y + c1.y);
      buf[i + 2 * h] = make_double2(a1.x - c1.x, a1.y - c1.y);
      buf[i + h] = make_double2(b1.x + d1.x, b1.y + d1.y);
      buf[i + 3 * h] = make_double2(b1.x - d1.x, b1.y - d1.y);
    }
    __syncthreads();
  }
  if (sh == logL) {  // the last stage, span L
    const int half = L >> 1, nb = TW * L / 2;
    for (int bf = threadIdx.x; bf < nb; bf += blockDim.x) {
      const int t = bf >> (logL - 1), pos = bf & (half - 1);
      const int i0 = t * L + pos, i1 = i0 + half;
      const double2 u = buf[i0], v = cmul(buf[i1], twiddle(tw, pos, cj));
      buf[i0] = make_double2(u.x + v.x, u.y + v.y);
      buf[i1] = make_double2(u.x - v.x, u.y - v.y);
    }
    __syncthreads();
  }
}

// decimation in frequency: natural order in, bit-reversed order out (the
// same transform as fft_dit).  Two stages per pass, spans 4h then 2h; an odd
// logL leaves the span-2 stage, whose twiddle is 1.  Ends with a barrier.
__device__ __forceinline__ void fft_dif(double2* buf, const double2* tw, int L, int logL, int TW, bool cj = false) {
  int sh = logL;
  for (; sh - 1 >= 1; sh -= 2) {
    const int h = 1 << (sh - 2), s1 = L >> sh, s2 = L >> (sh - 1), nq = TW * L / 4;
    for (int q = threadIdx.x; q < nq; q += blockDim.x) {
      const int t = q >> (logL - 2), r = q & ((L >> 2) - 1);
      const int pos = r & (h - 1), i = t * L + ((r >> (sh - 2)) << sh) + pos;
      const double2 a = buf[i], b = buf[i + h], c = buf[i + 2 * h], d = buf[i + 3 * h];
      const double2 a1 = make_double2(a.x + c.x, a.y + c.y);
      const double2 c1 = cmul(make_double2(a.x - c.x, a.y - c.y), twiddle(tw, pos * s1, cj));
      const double2 b1 = make_double2(b.x + d.x, b.y + d.y);
      const double2 d1 = cmul(make_double2(b.x - d.x, b.y - d.y), twiddle(tw, (pos + h) * s1, cj));
      const double2 w2 = twiddle(tw, pos * s2, cj);
      buf[i] = make_double2(a1.x + b1.x, a1.y + b1.y);
      buf[i + h] = cmul(make_double2(a1.x - b1.x, a1.y - b1.y), w2);
      buf[i + 2 * h] = make_double2(c1.x + d1.x, c1.y + d1.y);
      buf[i + 3 * h] = cmul(make_double2(c1.x - d1.x, c1.y - d1.y), w2);
    }
    __syncthreads();
  }
  if (sh == 1) {  // span 2
    const int nb = TW * L / 2;
    for (int bf = threadIdx.x; bf < nb; bf += blockDim.x) {
      const int i0 = 2 * bf, i1 = i0 + 1;
      const double2 u = buf[i0], v = buf[i1];
      buf[i0] = make_double2(u.x + v.x, u.y + v.y);
      buf[i1] = make_double2(u.x - v.x, u.y - v.y);
    }
    __syncthreads();
  }
}

// the L/2 twiddles of a table copied behind the lines in LDS when the plan
// left room for them (stw), else read where they are; the caller's barrier
// after its loads covers the copy
__device__ __forceinline__ const double2* stage_twiddles(double2* lds, const double2* __restrict__ tw, int L,
                                                         int stw) {
  if (!stw) return tw;
  for (int i = threadIdx.x; i < L / 2; i += blockDim.x) lds[i] = tw[i];
  return lds;
}

__device__ __forceinline__ int bit_rev(int k, int logL) {
  return logL == 0 ? 0 : (int)(__brev((unsigned)k) >> (32 - logL));
}

// TW lines of length L = 2^logL per workgroup; line t of group gi starts at
// (gi / per) A + (gi % per) TW C + t tstride and steps kstride (the kernel
// spectra at setup)
__global__ void __launch_bounds__(kBlock) fft_lines_kernel(double2* __restrict__ a, const double2* __restrict__ tw,
                                                           int L, int logL, int TW, int per, long long A, long long C,
                                                           long long tstride, long long kstride) {
  extern __shared__ double2 buf[];
  const int gi = blockIdx.x;
  const long long base = (long long)(gi / per) * A + (long long)(gi % per) * TW * C;
  const int tot = TW * L;
  const bool kfast = kstride == 1;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int t = kfast ? e / L : e % TW;
    const int k = kfast ? e % L : e / TW;
    buf[t * L + bit_rev(k, logL)] = a[base + t * tstride + k * kstride];
  }
  __syncthreads();
  fft_dit(buf, tw, L, logL, TW);
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int t = kfast ? e / L : e % TW;
    const int k = kfast ? e % L : e / TW;
    a[base + t * tstride + k * kstride] = buf[t * L + k];
  }
}

// rows: line ln = s n1 + t1 (ln < S n1) of pair q is row t1 of slab s
template <typename T>
__global__ void __launch_bounds__(kBlock) fft_rows_fwd_kernel(const double2* __restrict__ gin,
                                                              const typename cpx<T>::t* __restrict__ yin, int first,
                                                              Geometry g, FaceFFT ff) {
  extern __shared__ double2 buf[];
  const int q = blockIdx.y, f0 = 2 * q;
  const int n1 = g.face_n1[f0], n2 = g.face_n2[f0], R = g.R, B = g.batch;
  const int P1 = ff.P1[q], P2 = ff.P2[q], logL = ff.lg2[q], TW = ff.twr[q];
  const int nline = ff.S[q] * n1, ln0 = blockIdx.x * TW;
  if (ln0 >= nline) return;
  const int tot = TW * P2;
  const double2* tw = stage_twiddles(buf + tot, ff.tw + ff.twoff[q][0], P2, ff.stwr[q]);
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int t = e >> logL, k = e & (P2 - 1), ln = ln0 + t;
    double2 v = make_double2(0.0, 0.0);
    if (ln < nline && k < n2) {
      const int sl = ln / n1, t1 = ln - sl * n1;
      const int b = sl % B, l = (sl / B) % R, f = f0 + sl / (B * R);
      if (first) {
        v = gin[g.face_off[f] + (((long long)l * n1 + t1) * n2 + k) * B + b];
      } else {
        const auto yv = yin[face_point(g, f, l, t1, k) * B + b];
        v = make_double2((double)yv.x, (double)yv.y);
      }
    }
    buf[t * P2 + bit_rev(k, logL)] = v;
  }
  __syncthreads();
  fft_dit(buf, tw, P2, logL, TW);
  double2* W = ff.W + ff.woff[q];
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int t = e >> logL, k = e & (P2 - 1), ln = ln0 + t;
    if (ln < nline) {
      const int sl = ln / n1, t1 = ln - sl * n1;
      W[((long long)sl * P1 + t1) * P2 + k] = buf[t * P2 + k];
    }
  }
}

// columns: workgroup = (slab group side B + b, TW columns from c0); the R
// layers of the group sit in LDS one after the other ([l][t][k])
__global__ void __launch_bounds__(kBlock) fft_cols_kernel(Geometry g, FaceFFT ff) {
  extern __shared__ double2 buf[];
  const int q = blockIdx.y;
  const int n1 = g.face_n1[2 * q], R = g.R, B = g.batch;
  const int P1 = ff.P1[q], P2 = ff.P2[q], logL = ff.lg1[q], TW = ff.twc[q];
  const int per = P2 / TW;
  const int lgTW = __ffs(TW) - 1;  // TW is a power of two
  if ((int)blockIdx.x >= 2 * B * per) return;
  const int sg = blockIdx.x / per, c0 = (blockIdx.x % per) * TW;
  const int side = sg / B, b = sg % B;
  const int tot = TW * P1;
  const long long slab = (long long)P1 * P2;
  // forward twiddles along t1; the inverse ones are their conjugates
  const double2* tw = stage_twiddles(buf + R * tot, ff.tw + ff.twoff[q][2], P1, ff.stwc[q]);
  for (int l = 0; l < R; ++l) {
    const double2* src = ff.W + ff.woff[q] + (long long)((side * R + l) * B + b) * slab + c0;
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
      const int t = e & (TW - 1), k = e >> lgTW;
      buf[l * tot + t * P1 + bit_rev(k, logL)] = k < n1 ? src[(long long)k * P2 + t] : make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  fft_dit(buf, tw, P1, logL, R * TW);
  // Z(l) = sum_l' spec(l, l') W(l') / (P1 P2), point by point
  const double inv = 1.0 / (double)slab;
  const double2* spec = ff.spec + ff.soff[q];
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int t = e & (TW - 1), k = e >> lgTW;
    const long long m = (long long)k * P2 + c0 + t;
    double2 x[abc::kMaxR];
    for (int lp = 0; lp < R; ++lp) x[lp] = buf[lp * tot + t * P1 + k];
    for (int l = 0; l < R; ++l) {
      double zr = 0, zi = 0;
      for (int lp = 0; lp < R; ++lp) {
        const double2 kv = spec[(long long)(l * R + lp) * slab + m];
        zr += kv.x * x[lp].x - kv.y * x[lp].y;
        zi += kv.x * x[lp].y + kv.y * x[lp].x;
      }
      buf[l * tot + t * P1 + k] = make_double2(zr * inv, zi * inv);
    }
  }
  __syncthreads();
  fft_dif(buf, tw, P1, logL, R * TW, true);
  const int tout = TW * n1;
  for (int l = 0; l < R; ++l) {
    double2* dst = ff.Z + ff.woff[q] + (long long)((side * R + l) * B + b) * slab + c0;
    for (int e = threadIdx.x; e < tout; e += blockDim.x) {
      const int t = e & (TW - 1), k = e >> lgTW;
      dst[(long long)k * P2 + t] = buf[l * tot + t * P1 + bit_rev(k, logL)];
    }
  }
}

// inverse rows of Z (t1 < n1) and the face_kernel epilogue on t2 < n2
// mode 3 (shell stages of the one-pass sweep, one orbital): gout = alpha base +
// beta (B x + A E (yin + y2)), base and y2 optional
struct FaceAffine {
  const double2* base;
  const void* y2;
  double alpha, beta;
};

template <typename T, int R>
__global__ void __launch_bounds__(kBlock) fft_rows_inv_kernel(
    const double2* __restrict__ gin, double2* __restrict__ gout, double2* __restrict__ facc,
    double2* __restrict__ aux_out, const typename cpx<T>::t* __restrict__ yin, LocalBlock a, Geometry g, FaceFFT ff,
    double coef, int mode, int first, FaceAffine af) {
  extern __shared__ double2 buf[];
  const int q = blockIdx.y, f0 = 2 * q;
  const int n1 = g.face_n1[f0], n2 = g.face_n2[f0], B = g.batch;
  const int P1 = ff.P1[q], P2 = ff.P2[q], logL = ff.lg2[q], TW = ff.twr[q];
  const int nline = ff.S[q] * n1, ln0 = blockIdx.x * TW;
  if (ln0 >= nline) return;
  const double2* Z = ff.Z + ff.woff[q];
  const int tot = TW * P2;
  const double2* tw = stage_twiddles(buf + tot, ff.tw + ff.twoff[q][1], P2, ff.stwr[q]);
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int t = e >> logL, k = e & (P2 - 1), ln = ln0 + t;
    double2 v = make_double2(0.0, 0.0);
    if (ln < nline) {
      const int sl = ln / n1, t1 = ln - sl * n1;
      v = Z[((long long)sl * P1 + t1) * P2 + k];
    }
    buf[t * P2 + bit_rev(k, logL)] = v;
  }
  __syncthreads();
  fft_dit(buf, tw, P2, logL, TW);
  const int tout = TW * n2;
  for (int e = threadIdx.x; e < tout; e += blockDim.x) {
    const int t = e / n2, t2 = e - t * n2, ln = ln0 + t;
    if (ln >= nline) continue;
    const int sl = ln / n1, t1 = ln - sl * n1;
    const int b = sl % B, l = (sl / B) % R, f = f0 + sl / (B * R);
    const long long fe = g.face_off[f] + (((long long)l * n1 + t1) * n2 + t2) * B + b;
    const double2 cv = buf[t * P2 + t2];
    double sr = cv.x, si = cv.y;
    if (!first) {
      gout[fe] = make_double2(sr, si);
      continue;
    }
    if (mode == 3) {
      using C = typename cpx<T>::t;
      const C* y2 = static_cast<const C*>(af.y2);
      for (int lp = 0; lp < R; ++lp) {
        const double2 av = a.m[l * R + lp];
        const long long pp = face_point(g, f, lp, t1, t2);
        const auto yv = yin[pp];
        double yr = (double)yv.x, yi = (double)yv.y;
        if (y2) {
          const auto zv = y2[pp];
          yr += (double)zv.x;
          yi += (double)zv.y;
        }
        sr += av.x * yr - av.y * yi;
        si += av.x * yi + av.y * yr;
      }
      double2 o = make_double2(af.beta * sr, af.beta * si);
      if (af.base) {
        const double2 bv = af.base[fe];
        o.x += af.alpha * bv.x;
        o.y += af.alpha * bv.y;
      }
      gout[fe] = o;
      continue;
    }
    for (int lp = 0; lp < R; ++lp) {
      const double2 av = a.m[l * R + lp];
      const auto yv = yin[face_point(g, f, lp, t1, t2) * B + b];
      const double yr = (double)yv.x, yi = (double)yv.y;
      sr += av.x * yr - av.y * yi;
      si += av.x * yi + av.y * yr;
    }
    const double2 gn = make_double2(coef * sr, coef * si);
    if (mode == 0) {
      const double2 g0 = gin[fe];
      facc[fe] = make_double2(g0.x + gn.x, g0.y + gn.y);
      gout[fe] = gn;
    } else if (mode == 1) {
      double2 s2 = facc[fe];
      s2.x += gn.x;
      s2.y += gn.y;
      facc[fe] = s2;
      gout[fe] = gn;
    } else {
      const double2 s2 = facc[fe];
      aux_out[fe] = make_double2(s2.x + gn.x, s2.y + gn.y);
    }
  }
}

inline int ilog2(int v) {
  int k = 0;
  while ((1 << k) < v) ++k;
  return k;
}

// Lines per workgroup for transforms of length L over n lines: enough for
// every thread to own a butterfly (L TW / 2 >= kBlock), and no more, so that
// the few hundred lines of a face pair spread over many workgroups; the
// strided column pass takes at least `minTW` lines for wider segments.
inline int fft_lines_per_group(int L, int n, int minTW) {
  const int tw = std::max(std::max(1, 2 * kBlock / L), minTW);
  return std::min(n, std::min(tw, std::max(1, 4096 / L)));
}

// 2D transform of S slabs of P1 x P2 points at base, with the twiddle
// tables tw2 (length P2 lines) and tw1 (length P1 lines); at most 64 KB of
// LDS per workgroup (P <= 4096)
hipError_t fft2_slabs(double2* base, int P1, int P2, int S, const double2* tw2, const double2* tw1, hipStream_t st) {
  {
    const int L = P2, TW = fft_lines_per_group(L, P1, 1);
    fft_lines_kernel<<<S * P1 / TW, kBlock, (size_t)TW * L * sizeof(double2), st>>>(
        base, tw2, L, ilog2(L), TW, 1, (long long)TW * L, 0, L, 1);
  }
  {
    const int L = P1, TW = fft_lines_per_group(L, P2, 4);
    const int per = P2 / TW;
    fft_lines_kernel<<<S * per, kBlock, (size_t)TW * L * sizeof(double2), st>>>(
        base, tw1, L, ilog2(L), TW, per, (long long)P1 * P2, 1, 1, P2);
  }
  return hipGetLastError();
}

// the face operator of one stage by FFT: gout (first order: coef (B g + A E
// y) with the Taylor modes of face_kernel; zeroth: M E y)
template <typename T, int R>
hipError_t face_fft_apply(const abc_launch& L, const double2* gin, double2* gout, double2* facc, double2* aux_out,
                          const typename cpx<T>::t* yin, const LocalBlock& a, double coef, int mode, int first,
                          hipStream_t st, abc_timer* tm, const char* label, FaceAffine af = FaceAffine{}) {
  const FaceFFT& ff = *L.face_fft;
  const Geometry& g = L.g;
  unsigned nr = 0, nc = 0;
  size_t lr = 0, lc = 0;
  // threads: one per two points of the widest pair, whole waves, at most
  // kBlock (the four-point passes leave half of them idle, but the extra
  // waves hide more latency than the smaller blocks save: 204 against 215 us
  // per step at 128^3)
  int br = 64, bc = 64;
  for (int q = 0; q < 3; ++q) {
    const int n1 = g.face_n1[2 * q];
    br = std::max(br, std::min(kBlock, (ff.twr[q] * ff.P2[q] / 2 + 63) / 64 * 64));
    bc = std::max(bc, std::min(kBlock, (g.R * ff.twc[q] * ff.P1[q] / 2 + 63) / 64 * 64));
    nr = std::max(nr, (unsigned)((ff.S[q] * n1 + ff.twr[q] - 1) / ff.twr[q]));
    nc = std::max(nc, (unsigned)(2 * g.batch * (ff.P2[q] / ff.twc[q])));
    lr = std::max(lr, (size_t)(ff.twr[q] * ff.P2[q] + (ff.stwr[q] ? ff.P2[q] / 2 : 0)) * sizeof(double2));
    lc = std::max(lc, (size_t)(g.R * ff.twc[q] * ff.P1[q] + (ff.stwc[q] ? ff.P1[q] / 2 : 0)) * sizeof(double2));
  }
  fft_rows_fwd_kernel<T><<<dim3(nr, 3), br, lr, st>>>(gin, yin, first, g, ff);
  fft_cols_kernel<<<dim3(nc, 3), bc, lc, st>>>(g, ff);
  abc_launch_kernel_lds(tm, label, fft_rows_inv_kernel<T, R>, dim3(nr, 3), dim3(br), lr, st, gin, gout, facc,
                        aux_out, yin, a, g, ff, coef, mode, first, af);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// box form, one orbital: the same product with E y gathered once per stage
// into a contiguous vector x2, and kBoxRows rows per workgroup, so that every
// vector element a thread loads serves kBoxRows matrix rows.  Partial sums
// reduce within each wave by shuffles, then across the waves in LDS; the
// stage update is that of box_gemv_kernel.  Rows past nrow read the last row
// and write nothing.  Mode kGemvPlain writes the product itself (after the
// identity block's g for rows below ident).  The operator is streamed once
// per stage and read with nontemporal loads, so that it does not evict the
// vector from the caches (31^3, R = 3: 4.18 against 4.44 ms per first-order
// step, 6.1 to 6.5 TB/s)
// ---------------------------------------------------------------------------
constexpr int kBoxRows = 4, kBoxRowsMin = 4096;
constexpr int kGemvPlain = 3;
typedef double stream_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 stream_load(const double2* p) {
  const stream_d2 v = __builtin_nontemporal_load(reinterpret_cast<const stream_d2*>(p));
  return make_double2(v.x, v.y);
}

__global__ void __launch_bounds__(kBlock) box_gemv_rows_kernel(
    const double2* __restrict__ mat, int nrow, int naux, int ncol, int ident, const double2* __restrict__ gin,
    const double2* __restrict__ x2, double2* __restrict__ gout, double2* __restrict__ facc,
    double2* __restrict__ aux_out, double coef, int mode) {
  constexpr int RB = kBoxRows, NW = kBlock / 64;
  __shared__ double2 red[RB][NW];
  const int row0 = blockIdx.x * RB;
  const double2* mrow[RB];
  double sr[RB], si[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    mrow[r] = mat + (long long)min(row0 + r, nrow - 1) * ncol;
    sr[r] = si[r] = 0.0;
  }
  // boundary-variable columns; rows below ident skip them (their [0, I]
  // block is added in the update), and so does a workgroup of such rows
  for (int j = threadIdx.x; j < (row0 + RB > ident ? naux : 0); j += kBlock) {
    const double2 v = gin[j];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      if (row0 + r < ident) continue;
      const double2 m = stream_load(&mrow[r][j]);
      sr[r] += m.x * v.x - m.y * v.y;
      si[r] += m.x * v.y + m.y * v.x;
    }
  }
  // field columns
  for (int j = threadIdx.x; j < ncol - naux; j += kBlock) {
    const double2 v = x2[j];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const double2 m = stream_load(&mrow[r][naux + j]);
      sr[r] += m.x * v.x - m.y * v.y;
      si[r] += m.x * v.y + m.y * v.x;
    }
  }
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    for (int o = 32; o > 0; o >>= 1) {
      sr[r] += __shfl_down(sr[r], o, 64);
      si[r] += __shfl_down(si[r], o, 64);
    }
    if ((threadIdx.x & 63) == 0) red[r][threadIdx.x >> 6] = make_double2(sr[r], si[r]);
  }
  __syncthreads();
  if (threadIdx.x >= RB) return;
  const int r = threadIdx.x, row = row0 + r;
  if (row >= nrow) return;
  double2 t = red[r][0];
  for (int w = 1; w < NW; ++w) {
    t.x += red[r][w].x;
    t.y += red[r][w].y;
  }
  if (naux == 0) {
    gout[row] = t;
    return;
  }
  if (row < ident) {
    const double2 gv = gin[row + ident];
    t.x += gv.x;
    t.y += gv.y;
  }
  if (mode == kGemvPlain) {
    gout[row] = t;
    return;
  }
  const double2 gn = make_double2(coef * t.x, coef * t.y);
  if (mode == 0) {
    const double2 g0 = gin[row];
    facc[row] = make_double2(g0.x + gn.x, g0.y + gn.y);
    gout[row] = gn;
  } else if (mode == 1) {
    double2 sacc = facc[row];
    sacc.x += gn.x;
    sacc.y += gn.y;
    facc[row] = sacc;
    gout[row] = gn;
  } else {
    const double2 sacc = facc[row];
    aux_out[row] = make_double2(sacc.x + gn.x, sacc.y + gn.y);
  }
}

// ---------------------------------------------------------------------------
// box form: dense operator on Gamma.  One workgroup per row; the row of the
// rows x ncol matrix times [x1; x2] where x1 = the naux boundary variables of
// the stage (first and second order) or absent (naux = 0, zeroth), x2 = E y.
// out = coef * (row . x) with the stage update (naux > 0), or row . x.
// Rows below `ident` (second order: the n rows of df/dt) hold [0, I] on the
// boundary columns; they read only their E y columns and add g directly.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) box_gemv_kernel(
    const double2* __restrict__ mat, int naux, int ncol, int ident, const double2* __restrict__ gin,
    const typename cpx<T>::t* __restrict__ yin, const int* __restrict__ gamma_lin,
    double2* __restrict__ gout, double2* __restrict__ facc, double2* __restrict__ aux_out,
    int batch, double coef, int mode) {
  __shared__ double2 red[kBlock];
  const int row = blockIdx.x;
  const int b = blockIdx.y;
  double sr = 0, si = 0;
  const double2* mrow = mat + (long long)row * ncol;
  const int j0 = row < ident ? naux : 0;
  for (int j = j0 + threadIdx.x; j < ncol; j += blockDim.x) {
    const double2 m = mrow[j];
    double2 v;
    if (j < naux) {
      v = gin[(long long)j * batch + b];
    } else {
      const auto yv = yin[(long long)gamma_lin[j - naux] * batch + b];
      v = make_double2((double)yv.x, (double)yv.y);
    }
    sr += m.x * v.x - m.y * v.y;
    si += m.x * v.y + m.y * v.x;
  }
  red[threadIdx.x] = make_double2(sr, si);
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[threadIdx.x].x += red[threadIdx.x + s].x;
      red[threadIdx.x].y += red[threadIdx.x + s].y;
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const long long e = (long long)row * batch + b;
  if (naux == 0) {
    gout[e] = red[0];
    return;
  }
  if (row < ident) {
    const double2 gv = gin[(long long)(row + ident) * batch + b];
    red[0].x += gv.x;
    red[0].y += gv.y;
  }
  const double2 gn = make_double2(coef * red[0].x, coef * red[0].y);
  if (mode == 0) {
    const double2 g0 = gin[e];
    facc[e] = make_double2(g0.x + gn.x, g0.y + gn.y);
    gout[e] = gn;
  } else if (mode == 1) {
    double2 s = facc[e];
    s.x += gn.x;
    s.y += gn.y;
    facc[e] = s;
    gout[e] = gn;
  } else {
    const double2 s = facc[e];
    aux_out[e] = make_double2(s.x + gn.x, s.y + gn.y);
  }
}

// ---------------------------------------------------------------------------
// diagnostics: per-(orbital, block) partial sums, then a fixed-order finish
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 256;  // point blocks per orbital
constexpr int kAuxBlocks = 64;   // aux blocks per orbital

__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

template <typename T, int R, bool PER>
__global__ void __launch_bounds__(kBlock) diag_points_kernel(
    const typename cpx<T>::t* __restrict__ psi, const T* __restrict__ V, Geometry g, StencilCoef sc,
    int meanfield, double t0, double t3, double* __restrict__ part) {
  __shared__ double sh[kBlock];
  using C = typename cpx<T>::t;
  const int b = blockIdx.y, B = g.batch;
  double nrm = 0, en = 0, eint = 0;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < g.npts;
       p += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(p % g.nx);
    const int y = (int)((p / g.nx) % g.ny);
    const int z = (int)(p / ((long long)g.nx * g.ny));
    const C c0 = psi[p * B + b];
    const double cr = c0.x, ci = c0.y;
    double hr = sc.diag * cr, hi = sc.diag * ci;
    for (int k = 1; k <= R; ++k) {
      double ar = 0, ai = 0;
      int nb[6][3] = {{x + k, y, z}, {x - k, y, z}, {x, y + k, z}, {x, y - k, z}, {x, y, z + k}, {x, y, z - k}};
      for (int m = 0; m < 6; ++m) {
        int xx = nb[m][0], yy = nb[m][1], zz = nb[m][2];
        if (PER) {
          xx = (xx + g.nx) % g.nx; yy = (yy + g.ny) % g.ny; zz = (zz + g.nz) % g.nz;
        } else if (xx < 0 || xx >= g.nx || yy < 0 || yy >= g.ny || zz < 0 || zz >= g.nz) {
          continue;
        }
        const C v = psi[lin(g, xx, yy, zz) * B + b];
        ar += v.x;
        ai += v.y;
      }
      hr += sc.off[k] * ar;
      hi += sc.off[k] * ai;
    }
    if (V) {
      hr += (double)V[p] * cr;
      hi += (double)V[p] * ci;
    }
    nrm += cr * cr + ci * ci;
    en += cr * hr + ci * hi;
    if (meanfield && b == 0) {
      double rho = 0;
      for (int bb = 0; bb < B; ++bb) {
        const C v = psi[p * B + bb];
        rho += (double)v.x * v.x + (double)v.y * v.y;
      }
      eint += t0 * rho * rho / 2 + t3 * rho * rho * rho / 3;
    }
  }
  nrm = block_sum(nrm, sh);
  en = block_sum(en, sh);
  eint = block_sum(eint, sh);
  if (threadIdx.x == 0) {
    double* o = part + ((long long)b * (kRedBlocks + kAuxBlocks) + blockIdx.x) * 4;
    o[0] = nrm;
    o[1] = en;
    o[2] = eint;
    o[3] = 0;
  }
}

template <int R>
__global__ void __launch_bounds__(kBlock) diag_aux_kernel(const double2* __restrict__ aux, Geometry g,
                                                           LocalBlock q, long long nface_lines,
                                                           double* __restrict__ part) {
  // sum over face lines (f, t1, t2) of f^* q f per orbital
  __shared__ double sh[kBlock];
  const int b = blockIdx.y, B = g.batch;
  double s = 0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nface_lines;
       e += (long long)gridDim.x * blockDim.x) {
    // locate face f and transverse index
    long long acc = 0;
    int f = 0;
    for (; f < 6; ++f) {
      const long long m = (long long)g.face_n1[f] * g.face_n2[f];
      if (e < acc + m) break;
      acc += m;
    }
    const long long t = e - acc;
    const long long plane = (long long)g.face_n1[f] * g.face_n2[f];
    double2 v[R];
    for (int l = 0; l < R; ++l) v[l] = aux[g.face_off[f] + ((long long)l * plane + t) * B + b];
    for (int l = 0; l < R; ++l)
      for (int lp = 0; lp < R; ++lp) {
        const double2 qq = q.m[l * R + lp];
        // conj(v_l) * qq * v_lp, real part
        const double xr = qq.x * v[lp].x - qq.y * v[lp].y;
        const double xi = qq.x * v[lp].y + qq.y * v[lp].x;
        s += v[l].x * xr + v[l].y * xi;
      }
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    double* o = part + ((long long)b * (kRedBlocks + kAuxBlocks) + kRedBlocks + blockIdx.x) * 4;
    o[0] = s;
    o[1] = 0;
    o[2] = 0;
    o[3] = 0;
  }
}

__global__ void diag_box_aux_kernel(const double2* __restrict__ aux, const double2* __restrict__ qmat, int n,
                                    int batch, double* __restrict__ part) {
  // f^* Q f with dense Q (box form); rows strided over the aux blocks
  __shared__ double sh[kBlock];
  const int b = blockIdx.y;
  double s = 0;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    double xr = 0, xi = 0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      const double2 qq = qmat[(long long)i * n + j];
      const double2 v = aux[(long long)j * batch + b];
      xr += qq.x * v.x - qq.y * v.y;
      xi += qq.x * v.y + qq.y * v.x;
    }
    xr = block_sum(xr, sh);
    xi = block_sum(xi, sh);
    const double2 vi = aux[(long long)i * batch + b];
    s += vi.x * xr + vi.y * xi;
  }
  if (threadIdx.x == 0) {
    double* o = part + ((long long)b * (kRedBlocks + kAuxBlocks) + kRedBlocks + blockIdx.x) * 4;
    o[0] = s;
    o[1] = 0;
    o[2] = 0;
    o[3] = 0;
  }
}

__global__ void diag_finish_kernel(const double* __restrict__ part, int batch, double h3, int has_aux,
                                   double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const double* pb = part + (long long)b * (kRedBlocks + kAuxBlocks) * 4;
  double nrm = 0, en = 0, eint = 0, qa = 0;
  for (int i = 0; i < kRedBlocks; ++i) {
    nrm += pb[i * 4 + 0];
    en += pb[i * 4 + 1];
    eint += pb[i * 4 + 2];
  }
  if (has_aux)
    for (int i = 0; i < kAuxBlocks; ++i) qa += pb[(kRedBlocks + i) * 4];
  out[b] = h3 * nrm;
  out[batch + b] = h3 * (nrm + qa);
  out[2 * batch + b] = h3 * en;
  if (b == 0) out[3 * batch] = h3 * eint;
}

StencilCoef make_coef(const abc_launch& L) {
  StencilCoef sc{};
  const double s = 1.0 / (2.0 * L.h * L.h);
  sc.diag = -3.0 * L.c[0] * s;
  for (int k = 1; k <= L.g.R; ++k) sc.off[k] = -L.c[k] * s;
  return sc;
}

LocalBlock make_local(const double2* m) {
  LocalBlock a{};
  for (int i = 0; i < abc::kMaxR * abc::kMaxR; ++i) a.m[i] = m[i];
  return a;
}

// ---------------------------------------------------------------------------
// box form over an orbital batch: the operator is applied to all orbitals at
// once as a dense complex GEMM (rocBLAS zgemm, matrix cores) instead of one
// matrix pass per orbital.  gather: E y -> [gamma][orbital]; epilogue: the
// aux stage update of box_gemv_kernel on the GEMM result.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) box_gather_kernel(const typename cpx<T>::t* __restrict__ yin,
                                                            const int* __restrict__ gamma_lin, int n, int batch,
                                                            double2* __restrict__ out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * batch) return;
  const long long gi = e / batch;
  const int b = (int)(e - gi * batch);
  const auto v = yin[(long long)gamma_lin[gi] * batch + b];
  out[e] = make_double2((double)v.x, (double)v.y);
}

__global__ void __launch_bounds__(kBlock) box_epilogue_kernel(const double2* __restrict__ t,
                                                              const double2* __restrict__ gin,
                                                              double2* __restrict__ gout, double2* __restrict__ facc,
                                                              double2* __restrict__ aux_out, long long count,
                                                              double coef, int mode) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const double2 gn = make_double2(coef * t[e].x, coef * t[e].y);
  if (mode == 0) {
    const double2 g0 = gin[e];
    facc[e] = make_double2(g0.x + gn.x, g0.y + gn.y);
    gout[e] = gn;
  } else if (mode == 1) {
    double2 s2 = facc[e];
    s2.x += gn.x;
    s2.y += gn.y;
    facc[e] = s2;
    gout[e] = gn;
  } else {
    const double2 s2 = facc[e];
    aux_out[e] = make_double2(s2.x + gn.x, s2.y + gn.y);
  }
}

inline unsigned nblocks(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------------------
// Second order in the DtN maps' dominant subspace U (n x r, real), one
// orbital: a stage projects f, g and E y onto the subspace (one pass over U
// for the three vectors), applies the reduced operator [[0, I, A1~], [B0~,
// B1~, C~]] (two GEMVs: the constant [0, I] block is added, not read), lifts
// the two results back (one pass over U) and applies the stage update in the
// full coordinates, where the auxiliary variables stay.  The complex vectors ride in the
// products with U as rows of real matrices: column j of the packed 6 x n (or
// 4 x r) matrix holds the real and imaginary parts of the vectors' j-th
// entries.  The projection and the lift read U once each, in kernels of
// their own (the library GEMM took 0.3-0.8 ms for these 6- and 4-row shapes).
// ---------------------------------------------------------------------------

// W (6 x n, ld 6) from f = aux[0 .. n), g = aux[n .. 2n) and y
__global__ void __launch_bounds__(kBlock) pack3_kernel(double* __restrict__ W, const double2* __restrict__ aux,
                                                       const double2* __restrict__ y, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double2 f = aux[j], gg = aux[n + j], yy = y[j];
  double* w = W + 6LL * j;
  w[0] = f.x; w[1] = f.y; w[2] = gg.x; w[3] = gg.y; w[4] = yy.x; w[5] = yy.y;
}

// v = [f~; g~; y~] (3r complex) from Z (6 x r, ld 6)
__global__ void __launch_bounds__(kBlock) unpack3_kernel(double2* __restrict__ v, const double* __restrict__ Z,
                                                         int r) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= r) return;
  const double* z = Z + 6LL * j;
  v[j] = make_double2(z[0], z[1]);
  v[r + j] = make_double2(z[2], z[3]);
  v[2 * r + j] = make_double2(z[4], z[5]);
}

// Tp (4 x r, ld 4) from t = [t_f~; t_g~] (2r complex)
__global__ void __launch_bounds__(kBlock) pack2_kernel(double* __restrict__ Tp, const double2* __restrict__ t, int r) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= r) return;
  const double2 a = t[j], b = t[r + j];
  double* q = Tp + 4LL * j;
  q[0] = a.x; q[1] = a.y; q[2] = b.x; q[3] = b.y;
}

// Z (6 x r, ld 6) = W (6 x n, ld 6) U (n x r, column-major): a workgroup
// takes kProjCols columns of U, its threads stride over the n rows (each U
// column read once, coalesced); the partial sums are reduced within each
// wave by shuffles and across the waves in LDS, in a fixed order
constexpr int kProjCols = 8;
__global__ void __launch_bounds__(kBlock) proj_kernel(const double* __restrict__ U, int n, int r,
                                                      const double* __restrict__ W, double* __restrict__ Z) {
  constexpr int NV = kProjCols * 6, NW = kBlock / 64;
  __shared__ double red[NW][NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j0 = blockIdx.x * kProjCols;
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) {
    double w[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) w[c] = W[6LL * i + c];
#pragma unroll
    for (int q = 0; q < kProjCols; ++q) {
      const double u = j0 + q < r ? U[(long long)(j0 + q) * n + i] : 0.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) acc[q * 6 + c] += w[c] * u;
    }
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double v = acc[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wv][q] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < NV) {
    const int q = threadIdx.x;
    double sum = red[0][q];
#pragma unroll
    for (int k = 1; k < NW; ++k) sum += red[k][q];
    const int j = j0 + q / 6;
    if (j < r) Z[6LL * j + q % 6] = sum;
  }
}

// Tl (4 x n, ld 4) = Tp (4 x r, ld 4) U^T from the row-major copy Ut of U:
// a wave takes kLiftRows rows i of Ut and its lanes stride the r columns
// (coalesced rows, streamed once; each Tp entry serves the wave's rows); the
// four sums of each row reduce over the wave by shuffles in a fixed order
constexpr int kLiftRows = 4;
__global__ void __launch_bounds__(kBlock) lift_kernel(const double* __restrict__ Ut, int n, int r,
                                                      const double* __restrict__ Tp, double* __restrict__ Tl) {
  const int lane = threadIdx.x & 63;
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const long long i0 = wave * kLiftRows;
  if (i0 >= n) return;  // whole waves
  const double* row[kLiftRows];
#pragma unroll
  for (int k = 0; k < kLiftRows; ++k) row[k] = Ut + min(i0 + k, (long long)n - 1) * r;
  double acc[kLiftRows][4];
#pragma unroll
  for (int k = 0; k < kLiftRows; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[k][c] = 0.0;
  for (int j = lane; j < r; j += 64) {
    const double2 t01 = *reinterpret_cast<const double2*>(Tp + 4LL * j);
    const double2 t23 = *reinterpret_cast<const double2*>(Tp + 4LL * j + 2);
#pragma unroll
    for (int k = 0; k < kLiftRows; ++k) {
      const double u = row[k][j];
      acc[k][0] += t01.x * u;
      acc[k][1] += t01.y * u;
      acc[k][2] += t23.x * u;
      acc[k][3] += t23.y * u;
    }
  }
#pragma unroll
  for (int k = 0; k < kLiftRows; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc[k][c] += __shfl_down(acc[k][c], off, 64);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kLiftRows; ++k)
      if (i0 + k < n)
#pragma unroll
        for (int c = 0; c < 4; ++c) Tl[4 * (i0 + k) + c] = acc[k][c];
  }
}

// the stage update of box_epilogue_kernel on T = [T_f; T_g] read from the
// lifted 4 x n matrix (element e: part e / n, entry e % n)
__global__ void __launch_bounds__(kBlock) lifted_epilogue_kernel(const double* __restrict__ Tl,
                                                                 const double2* __restrict__ gin,
                                                                 double2* __restrict__ gout,
                                                                 double2* __restrict__ facc,
                                                                 double2* __restrict__ aux_out, int n, double coef,
                                                                 int mode) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2LL * n) return;
  const int part = (int)(e / n), j = (int)(e % n);
  const double* q = Tl + 4LL * j + 2 * part;
  const double2 gn = make_double2(coef * q[0], coef * q[1]);
  if (mode == 0) {
    const double2 g0 = gin[e];
    facc[e] = make_double2(g0.x + gn.x, g0.y + gn.y);
    gout[e] = gn;
  } else if (mode == 1) {
    double2 s2 = facc[e];
    s2.x += gn.x;
    s2.y += gn.y;
    facc[e] = s2;
    gout[e] = gn;
  } else {
    const double2 s2 = facc[e];
    aux_out[e] = make_double2(s2.x + gn.x, s2.y + gn.y);
  }
}

template <typename T>
hipError_t second_reduced_stage(const abc_launch& L, const abc_scratch& S, const typename cpx<T>::t* ycur,
                                const double2* gcur, double2* gnext, double2* aux, double coef, int mode,
                                hipStream_t st, abc_timer* tm, const char* label) {
  const int n = L.n_gamma, r = L.box_r;
  double* W = S.bpack;  // 6 x n in, then the lifted 4 x n
  double* Z = S.bred;   // 6 x r
  double2* v = reinterpret_cast<double2*>(S.bred + 6LL * r);  // [f~; g~; y~]
  double2* t = v + 3LL * r;                                      // [t_f~; t_g~]
  double* Tp = reinterpret_cast<double*>(t + 2LL * r);           // 4 x r
  abc_launch_kernel(tm, label, box_gather_kernel<T>, dim3(nblocks(n)), dim3(kBlock), st, ycur, L.gamma_lin, n, 1,
                    S.bwork[0]);
  abc_launch_kernel(tm, "reduced_pack", pack3_kernel, dim3(nblocks(n)), dim3(kBlock), st, W, gcur,
                    (const double2*)S.bwork[0], n);
  abc_launch_kernel(tm, "reduced_project", proj_kernel, dim3((unsigned)((r + kProjCols - 1) / kProjCols)),
                    dim3(kBlock), st, L.box_U, n, r, (const double*)W, Z);
  abc_launch_kernel(tm, "reduced_unpack", unpack3_kernel, dim3(nblocks(r)), dim3(kBlock), st, v, (const double*)Z, r);
  // t_g~ = [B0~ B1~ C~] v (rows r .. 2r of the row-major operator);
  // t_f~ = g~ + A1~ y~ (rows 0 .. r: their [0, I] block on the columns
  // 0 .. 2r is not read, g~ is added)
  const int ld = 3 * r;
  const unsigned rb = (unsigned)((r + kBoxRows - 1) / kBoxRows);
  abc_launch_kernel(tm, "reduced_operator", box_gemv_rows_kernel, dim3(rb), dim3(kBlock), st,
                    (const double2*)(L.box_red + (long long)r * ld), r, 0, ld, 0, (const double2*)nullptr,
                    (const double2*)v, t + r, (double2*)nullptr, (double2*)nullptr, 0.0, kGemvPlain);
  abc_launch_kernel(tm, "reduced_operator", box_gemv_rows_kernel, dim3(rb), dim3(kBlock), st,
                    (const double2*)L.box_red, r, 2 * r, ld, r, (const double2*)v, (const double2*)(v + 2LL * r), t,
                    (double2*)nullptr, (double2*)nullptr, 0.0, kGemvPlain);
  abc_launch_kernel(tm, "reduced_pack", pack2_kernel, dim3(nblocks(r)), dim3(kBlock), st, Tp, (const double2*)t, r);
  const long long lift_threads = (long long)(n + kLiftRows - 1) / kLiftRows * 64;
  abc_launch_kernel(tm, "reduced_lift", lift_kernel, dim3((unsigned)((lift_threads + kBlock - 1) / kBlock)),
                    dim3(kBlock), st, L.box_Ut, n, r, (const double*)Tp, W);
  abc_launch_kernel(tm, "box_epilogue", lifted_epilogue_kernel, dim3(nblocks(2LL * n)), dim3(kBlock), st,
                    (const double*)W, gcur, gnext, S.facc, aux, n, coef, mode);
  return hipGetLastError();
}

// Box form over an orbital batch: T = Op X, complex FP64, on the matrix cores.
// Op is the row-major operator (rows x ld); X = [X1; X2] stacks the
// auxiliary input (na rows, [row][orbital]) on the gathered E y (ld - na
// rows); T is [row][orbital].  Complex products as three real products
// (below) with v_mfma_f64_16x16x4f64, which computes
// D (16 x 16) += A (16 x 4) B (4 x 16) over the wave: lane l holds A[l % 16][l / 16],
// B[l / 16][l % 16] and, in its v-th result register, D[l / 16 + 4 v][l % 16].
// A workgroup owns 16 operator rows and all orbitals (NT tiles of 16
// columns); its kGemmSplit waves take every kGemmSplit-th chunk of 16 k
// and their partial products are summed in LDS in wave order
// (deterministic).  When the row tiles alone would leave part of the chip
// idle in the last round of workgroups, K is further split over ks
// workgroups per row tile (blockIdx.y), each writing its partial product,
// and a second kernel adds the ks partials in order.  In a chunk each lane loads four consecutive
// operator entries of its row (64 B): k quad kq = l / 16 takes entries
// 4 kq .. 4 kq + 3, and MFMA j uses entry 4 kq + j (the sum over k is the
// same in any order; A and B use the same one).  The operator is streamed
// once per stage for all orbitals; X (K x nb) stays in L2.
constexpr int kGemmSplit = 8;
constexpr int kGemmMaxKs = 4;  // workgroups per row tile at most
typedef double gemm_d4 __attribute__((ext_vector_type(4)));

template <int NT>
__global__ void __launch_bounds__(64 * kGemmSplit) box_gemm_kernel(const double2* __restrict__ op, int rows, int ld,
                                                                  int na, const double2* __restrict__ x1,
                                                                  const double2* __restrict__ x2, int nb,
                                                                  double2* __restrict__ t) {
  __shared__ double2 red[kGemmSplit][NT][4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row0 = blockIdx.x * 16;
  const int ar = lane & 15, kq = lane >> 4;
  const int arow = row0 + ar;
  const bool arow_ok = arow < rows;
  const double2* oprow = op + (long long)(arow_ok ? arow : 0) * ld;
  const int ks = gridDim.y, ksi = blockIdx.y;  // K split over workgroups
  t += (long long)ksi * rows * nb;
  // three real products per complex product (Karatsuba): with Op = a + ib
  // and X = c + id, p1 = (a + b) c, p2 = a (d - c), p3 = b (c + d), and
  // Re T = p1 - p3, Im T = p1 + p2
  gemm_d4 p1[NT], p2[NT], p3[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) p1[u] = p2[u] = p3[u] = gemm_d4{0, 0, 0, 0};
  for (int k0 = 16 * (ksi * kGemmSplit + w); k0 < ld; k0 += 16 * kGemmSplit * ks) {
    double2 a[4];
    double2 b[NT][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + 4 * kq + j;
      a[j] = (arow_ok && k < ld) ? oprow[k] : make_double2(0, 0);
      const double2* xr = k < na ? x1 + (long long)k * nb : x2 + (long long)(k - na) * nb;
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        const int col = u * 16 + ar;
        b[u][j] = (k < ld && col < nb) ? xr[col] : make_double2(0, 0);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double apb = a[j].x + a[j].y;
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        p1[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(apb, b[u][j].x, p1[u], 0, 0, 0);
        p2[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j].x, b[u][j].y - b[u][j].x, p2[u], 0, 0, 0);
        p3[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j].y, b[u][j].x + b[u][j].y, p3[u], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[w][u][v][lane] = make_double2(p1[u][v] - p3[u][v], p1[u][v] + p2[u][v]);
  __syncthreads();
  // the waves' partial sums in a fixed order; element e = (u, v, lane)
  for (int e = threadIdx.x; e < NT * 4 * 64; e += 64 * kGemmSplit) {
    const int u = e >> 8, v = (e >> 6) & 3, l = e & 63;
    double2 sum = red[0][u][v][l];
#pragma unroll
    for (int q = 1; q < kGemmSplit; ++q) {
      const double2 p = red[q][u][v][l];
      sum.x += p.x;
      sum.y += p.y;
    }
    const int row = row0 + (l >> 4) + 4 * v, col = u * 16 + (l & 15);
    if (row < rows && col < nb) t[(long long)row * nb + col] = sum;
  }
}

// t[e] = sum over the ks partial products, in order
__global__ void __launch_bounds__(kBlock) box_gemm_reduce_kernel(const double2* __restrict__ part, int ks,
                                                                 long long cnt, double2* __restrict__ t) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= cnt) return;
  double2 s = part[e];
  for (int q = 1; q < ks; ++q) {
    const double2 p = part[(long long)q * cnt + e];
    s.x += p.x;
    s.y += p.y;
  }
  t[e] = s;
}

// workgroups per row tile: the split (up to kGemmMaxKs, keeping at least two
// chunks of 16 k per wave) whose last round of workgroups leaves the fewest
// compute units idle; 1 unless that gains more than 2 %
int gemm_k_split(int rows, int ld) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || n < 1)
      n = 256;
    cus = n;
  }
  const long long tiles = (rows + 15) / 16, chunks = (ld + 15) / 16;
  int best = 1;
  double best_eff = (double)tiles / (double)(((tiles + cus - 1) / cus) * cus);
  for (int ks = 2; ks <= kGemmMaxKs; ++ks) {
    if (chunks < 2LL * kGemmSplit * ks) break;
    const long long wg = tiles * ks;
    const double eff = (double)wg / (double)(((wg + cus - 1) / cus) * cus);
    if (eff > best_eff + 0.02) {
      best_eff = eff;
      best = ks;
    }
  }
  return best;
}

// T = Op [X1; X2] for nb <= 64 orbitals (one to four column tiles); part
// (box_gemm_part_elems(rows nb) elements, or null) holds the partial
// products when K is split over workgroups
hipError_t box_gemm(abc_timer* tm, const double2* op, int rows, int ld, int na, const double2* x1,
                    const double2* x2, int nb, double2* t, double2* part, hipStream_t st) {
  const int ks = part ? gemm_k_split(rows, ld) : 1;
  const dim3 g((unsigned)((rows + 15) / 16), (unsigned)ks), b(64 * kGemmSplit);
  const int nt = (nb + 15) / 16;
  double2* out = ks > 1 ? part : t;
  if (nt == 1) abc_launch_kernel(tm, "box_gemm", box_gemm_kernel<1>, g, b, st, op, rows, ld, na, x1, x2, nb, out);
  else if (nt == 2) abc_launch_kernel(tm, "box_gemm", box_gemm_kernel<2>, g, b, st, op, rows, ld, na, x1, x2, nb, out);
  else if (nt == 3) abc_launch_kernel(tm, "box_gemm", box_gemm_kernel<3>, g, b, st, op, rows, ld, na, x1, x2, nb, out);
  else if (nt == 4) abc_launch_kernel(tm, "box_gemm", box_gemm_kernel<4>, g, b, st, op, rows, ld, na, x1, x2, nb, out);
  else return hipErrorInvalidValue;
  if (ks > 1) {
    const long long cnt = (long long)rows * nb;
    abc_launch_kernel(tm, "box_gemm_sum", box_gemm_reduce_kernel, dim3((unsigned)((cnt + kBlock - 1) / kBlock)),
                      dim3(kBlock), st, (const double2*)part, ks, cnt, t);
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Boundary shell of the one-pass sweep with a non-local face operator (first
// order, face form, window > 0 or exact sections; one orbital).
//
// The step is linear in (psi, f).  Split every stage quantity of the factored
// step (t, v, s, u') into the box with zero boundary values (the "Dirichlet
// chain", what the one-pass sweep without a condition computes) plus a
// correction delta driven by the E^T f terms.  delta_t lives on the face
// layers only and every later stage widens it by R layers, so delta_u'
// vanishes deeper than 4R: the step is the plain sweep plus delta_u' on a
// shell of depth 4R.  The auxiliary stages need the full stage values on the
// face layers (Dirichlet chain + delta), and the Dirichlet chain there needs
// psi only 4R deep.  So after the condition-free sweep, four small rounds
// compute, on shells of shrinking (Dirichlet) and growing (delta) depth,
// everything the boundary needs, with one application of the face operator
// B per round; the last adds delta_u' to the swept state.  Stage formulas (D = dt, L_psi(y, g) =
// -i (H y + E^T g), L_f(y, g) = B g + A E y):
//   round 1: t_D = a1 psi + b1 D L_psi(psi)        depth < 3R
//            dt  = b1 D L_psi(0, f)                 depth < R
//            t_f = a1 f + b1 D L_f(psi, f)
//   round 2: v_D = psi + D L_psi(t_D)               depth < 2R
//            dv  = D L_psi(dt, t_f)                 depth < 2R
//            v_f = f + D L_f(t_D + dt, t_f)
//   round 3: s_D = a2 v_D + b2 D L_psi(v_D)         depth < R
//            ds  = a2 dv + b2 D L_psi(dv, v_f)      depth < 3R
//            s_f = a2 v_f + b2 D L_f(v_D + dv, v_f)
//   round 4: du  = dv + D L_psi(ds, s_f)            depth < 4R
//            f'  = v_f + D L_f(s_D + ds, s_f)
// ---------------------------------------------------------------------------

// points of depth < d (distance to the nearest face), as six disjoint
// blocks: the x slabs whole, the y slabs between them, the z slabs inside
// both
struct ShellBox {
  int d, xl, xh, yl, yh, zl, zh, mx, my;
  long long off[7];
  unsigned blk[7];  // first workgroup of each block: a workgroup stays in one block
};

ShellBox make_shell_box(const Geometry& g, int d) {
  ShellBox b{};
  b.d = d;
  b.xl = std::min(d, g.nx);
  b.xh = std::min(d, g.nx - b.xl);
  b.mx = g.nx - b.xl - b.xh;
  b.yl = std::min(d, g.ny);
  b.yh = std::min(d, g.ny - b.yl);
  b.my = g.ny - b.yl - b.yh;
  b.zl = std::min(d, g.nz);
  b.zh = std::min(d, g.nz - b.zl);
  const long long cnt[6] = {(long long)b.xl * g.ny * g.nz, (long long)b.xh * g.ny * g.nz,
                            (long long)b.mx * b.yl * g.nz, (long long)b.mx * b.yh * g.nz,
                            (long long)b.mx * b.my * b.zl, (long long)b.mx * b.my * b.zh};
  b.off[0] = 0;
  b.blk[0] = 0;
  for (int i = 0; i < 6; ++i) {
    b.off[i + 1] = b.off[i] + cnt[i];
    b.blk[i + 1] = b.blk[i] + (unsigned)((cnt[i] + kBlock - 1) / kBlock);
  }
  return b;
}

// Coordinates of the shell point of thread t in workgroup wg (relative to the
// stage's first workgroup); false past the end of the workgroup's block.  The
// block, its sizes and offsets are wave-uniform (scalar), so the decode costs
// two 32-bit divisions and no per-lane access to the argument struct.
__device__ __forceinline__ bool shell_point(const Geometry& g, const ShellBox& b, unsigned wg, unsigned t, int& x,
                                           int& y, int& z) {
  int r = 0;
#pragma unroll
  for (int k = 1; k < 6; ++k) r += wg >= b.blk[k] ? 1 : 0;
  const unsigned q = (wg - b.blk[r]) * kBlock + t;
  if (q >= (unsigned)(b.off[r + 1] - b.off[r])) return false;
  // inner width (fastest), middle extent, offsets of the three coordinates
  unsigned wi, wm;
  int ox, oy, oz;
  if (r < 2) {
    wi = r == 0 ? b.xl : b.xh;
    wm = g.ny;
    ox = r == 0 ? 0 : g.nx - b.xh;
    oy = 0;
    oz = 0;
  } else if (r < 4) {
    wi = b.mx;
    wm = r == 2 ? b.yl : b.yh;
    ox = b.xl;
    oy = r == 2 ? 0 : g.ny - b.yh;
    oz = 0;
  } else {
    wi = b.mx;
    wm = b.my;
    ox = b.xl;
    oy = b.yl;
    oz = r == 4 ? 0 : g.nz - b.zh;
  }
  const unsigned row = q / wi;
  const unsigned zz = row / wm;
  x = (int)(q - row * wi) + ox;
  y = (int)(row - zz * wm) + oy;
  z = (int)zz + oz;
  return true;
}

__device__ __forceinline__ int point_depth(const Geometry& g, int x, int y, int z) {
  return min(min(min(x, g.nx - 1 - x), min(y, g.ny - 1 - y)), min(z, g.nz - 1 - z));
}

// one shell stage: out = alpha base + beta (-i) (H in + E^T aux) on the
// points of depth < box.d, or out += that with accumulate.  in and base read
// as zero outside the box and at depth >= in_depth / base_depth (where they
// are zero by construction and their buffers hold nothing); null pointers
// are zero.  FP64 arithmetic.
template <typename C>
struct ShellStage {
  ShellBox box;
  const C* in;
  const C* base;
  const double2* aux;
  C* out;
  int in_depth, base_depth, accumulate;
  double alpha, beta;
  unsigned nblk;
};

template <typename T, int R>
__device__ __forceinline__ void shell_stage_point(const ShellStage<typename cpx<T>::t>& sp, unsigned wg,
                                                  const Geometry& g, const T* __restrict__ V, StencilCoef sc) {
  using C = typename cpx<T>::t;
  int x, y, z;
  if (!shell_point(g, sp.box, wg, threadIdx.x, x, y, z)) return;
  const int p = (z * g.ny + y) * g.nx + x;
  // The neighbour loads read valid addresses (clamped coordinates; an absent
  // input reads the output array) and are masked afterwards, all issued
  // before the first use.
  const bool has_in = sp.in != nullptr, has_aux = sp.aux != nullptr, has_base = sp.base != nullptr;
  const C* in = has_in ? sp.in : sp.out;
  const bool masked = sp.in_depth <= sp.box.d + R;  // neighbours deeper than in_depth exist
  int nidx[1 + 6 * R];
  bool nok[1 + 6 * R];
  auto nb_at = [&](int m, int xx, int yy, int zz) {
    const bool inb = (unsigned)xx < (unsigned)g.nx && (unsigned)yy < (unsigned)g.ny && (unsigned)zz < (unsigned)g.nz;
    const int cx = min(max(xx, 0), g.nx - 1), cy = min(max(yy, 0), g.ny - 1), cz = min(max(zz, 0), g.nz - 1);
    nidx[m] = (cz * g.ny + cy) * g.nx + cx;
    nok[m] = has_in && inb && (!masked || point_depth(g, cx, cy, cz) < sp.in_depth);
  };
  nb_at(0, x, y, z);
#pragma unroll
  for (int k = 1; k <= R; ++k) {
    nb_at(6 * k - 5, x - k, y, z);
    nb_at(6 * k - 4, x + k, y, z);
    nb_at(6 * k - 3, x, y - k, z);
    nb_at(6 * k - 2, x, y + k, z);
    nb_at(6 * k - 1, x, y, z - k);
    nb_at(6 * k, x, y, z + k);
  }
  C nv[1 + 6 * R];
#pragma unroll
  for (int m = 0; m < 1 + 6 * R; ++m) nv[m] = in[nidx[m]];
  const double vp = V ? (double)V[p] : 0.0;
  // the rest only where it is used (the loads come from L2 with little
  // reuse, so their number, not their latency, sets the time): the base and
  // the accumulated output by the stage's (uniform) flags, the face values
  // on the face layers only
  C bv{}, ov{};
  if (has_base) bv = sp.base[p];
  if (sp.accumulate) ov = sp.out[p];
  double2 v0{}, v1{}, v2{}, v3{}, v4{}, v5{};
  const bool on_faces = has_aux && point_depth(g, x, y, z) < R;
  if (on_faces) {
    // E^T aux: the six faces, layer clamped to [0, R) and masked below
    const int lx0 = min(x, R - 1), lx1 = min(g.nx - 1 - x, R - 1);
    const int ly0 = min(y, R - 1), ly1 = min(g.ny - 1 - y, R - 1);
    const int lz0 = min(z, R - 1), lz1 = min(g.nz - 1 - z, R - 1);
    auto fv = [&](int f, int l, int t1, int t2) {
      return sp.aux[g.face_off[f] + ((long long)l * g.face_n1[f] + t1) * g.face_n2[f] + t2];
    };
    v0 = fv(0, lx0, z, y);
    v1 = fv(1, lx1, z, y);
    v2 = fv(2, ly0, z, x);
    v3 = fv(3, ly1, z, x);
    v4 = fv(4, lz0, y, x);
    v5 = fv(5, lz1, y, x);
  }
  // -- arithmetic
  double hr = 0, hi = 0;
  if (has_in) {
    const double dg = sc.diag + vp;
    hr = nok[0] ? dg * (double)nv[0].x : 0.0;
    hi = nok[0] ? dg * (double)nv[0].y : 0.0;
#pragma unroll
    for (int k = 1; k <= R; ++k) {
      double sx = 0, sy = 0;
#pragma unroll
      for (int m = 6 * k - 5; m <= 6 * k; ++m) {
        sx += nok[m] ? (double)nv[m].x : 0.0;
        sy += nok[m] ? (double)nv[m].y : 0.0;
      }
      hr += sc.off[k] * sx;
      hi += sc.off[k] * sy;
    }
  }
  if (on_faces) {
    const bool m0 = x < R, m1 = x >= g.nx - R, m2 = y < R, m3 = y >= g.ny - R, m4 = z < R, m5 = z >= g.nz - R;
    hr += (m0 ? v0.x : 0.0) + (m1 ? v1.x : 0.0) + (m2 ? v2.x : 0.0) + (m3 ? v3.x : 0.0) + (m4 ? v4.x : 0.0) +
          (m5 ? v5.x : 0.0);
    hi += (m0 ? v0.y : 0.0) + (m1 ? v1.y : 0.0) + (m2 ? v2.y : 0.0) + (m3 ? v3.y : 0.0) + (m4 ? v4.y : 0.0) +
          (m5 ? v5.y : 0.0);
  }
  // -i (hr + i hi) = hi - i hr
  double orr = sp.beta * hi, oi = -sp.beta * hr;
  if (has_base && point_depth(g, x, y, z) < sp.base_depth) {
    orr += sp.alpha * (double)bv.x;
    oi += sp.alpha * (double)bv.y;
  }
  if (sp.accumulate) {
    orr += (double)ov.x;
    oi += (double)ov.y;
  }
  C o;
  o.x = (T)orr;
  o.y = (T)oi;
  sp.out[p] = o;
}

// two independent shell stages in one launch (blocks [0, a.nblk) run a)
template <typename T, int R>
__global__ void __launch_bounds__(kBlock) shell_stage_kernel(ShellStage<typename cpx<T>::t> a,
                                                             ShellStage<typename cpx<T>::t> b, Geometry g,
                                                             const T* __restrict__ V, StencilCoef sc) {
  if (blockIdx.x < a.nblk)
    shell_stage_point<T, R>(a, blockIdx.x, g, V, sc);
  else
    shell_stage_point<T, R>(b, blockIdx.x - a.nblk, g, V, sc);
}

// face operator of a shell round (one orbital, any window):
// out = alpha base + beta (sum_{|p| <= w} k(p) x + A E (y + y2))
template <typename T, int R>
__global__ void __launch_bounds__(kBlock) face_affine_kernel(const double2* __restrict__ xin,
                                                             double2* __restrict__ out,
                                                             const typename cpx<T>::t* __restrict__ yin,
                                                             const double2* __restrict__ ker, LocalBlock a, Geometry g,
                                                             int w, FaceAffine af) {
  using C = typename cpx<T>::t;
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= g.face_off[6]) return;
  int f = 0;
  while (e >= g.face_off[f + 1]) ++f;
  const long long r = e - g.face_off[f];
  const int n1 = g.face_n1[f], n2 = g.face_n2[f];
  const int t2 = (int)(r % n2);
  const int t1 = (int)((r / n2) % n1);
  const int l = (int)(r / ((long long)n1 * n2));
  const int K = 2 * w + 1;
  double sr = 0, si = 0;
  const int j1lo = max(0, t1 - w), j1hi = min(n1 - 1, t1 + w);
  const int j2lo = max(0, t2 - w), j2hi = min(n2 - 1, t2 + w);
  for (int lp = 0; lp < R; ++lp) {
    const double2* kl = ker + ((long long)(l * R + lp)) * K * K;
    const double2* xl = xin + g.face_off[f] + (long long)lp * n1 * n2;
    for (int j1 = j1lo; j1 <= j1hi; ++j1) {
      const double2* krow = kl + (long long)(t1 - j1 + w) * K;
      for (int j2 = j2lo; j2 <= j2hi; ++j2) {
        const double2 kv = krow[t2 - j2 + w];
        const double2 v = xl[(long long)j1 * n2 + j2];
        sr += kv.x * v.x - kv.y * v.y;
        si += kv.x * v.y + kv.y * v.x;
      }
    }
  }
  const C* y2 = static_cast<const C*>(af.y2);
  for (int lp = 0; lp < R; ++lp) {
    const double2 av = a.m[l * R + lp];
    const long long pp = face_point(g, f, lp, t1, t2);
    const C yv = yin[pp];
    double yr = (double)yv.x, yi = (double)yv.y;
    if (y2) {
      const C zv = y2[pp];
      yr += (double)zv.x;
      yi += (double)zv.y;
    }
    sr += av.x * yr - av.y * yi;
    si += av.x * yi + av.y * yr;
  }
  double2 o = make_double2(af.beta * sr, af.beta * si);
  if (af.base) {
    const double2 bv = af.base[e];
    o.x += af.alpha * bv.x;
    o.y += af.alpha * bv.y;
  }
  out[e] = o;
}

// The same, tiled: a workgroup computes kAT1 x kAT2 outputs of one face
// layer; the inputs it needs ((kAT1 + 2w) x (kAT2 + 2w) per source layer,
// zero outside the face) and the taps are staged in dynamic LDS once.  Each
// thread owns four consecutive outputs of a row and every kASplit-th tap
// row, and slides a four-wide input window along each tap row, so one tap
// and one new input (two LDS reads) feed four complex multiply-adds; the
// kASplit partial sums are added in LDS.
constexpr int kAT1 = 8, kAT2 = 32, kASplit = 8, kABlock = kAT1 * (kAT2 / 4) * kASplit;  // 512 threads
inline size_t face_affine_lds(int R, int w) {
  const int K = 2 * w + 1;
  return ((size_t)R * (kAT1 + 2 * w) * (kAT2 + 2 * w) + (size_t)R * K * K + (size_t)(kASplit - 1) * kAT1 * kAT2) *
         sizeof(double2);
}
inline bool face_affine_tiled_ok(int R, int w) { return w >= 2 && face_affine_lds(R, w) <= 64 * 1024; }

template <typename T, int R>
__global__ void __launch_bounds__(kABlock) face_affine_tiled_kernel(const double2* __restrict__ xin,
                                                                    double2* __restrict__ out,
                                                                    const typename cpx<T>::t* __restrict__ yin,
                                                                    const double2* __restrict__ ker, LocalBlock a,
                                                                    Geometry g, int w, FaceAffine af) {
  using C = typename cpx<T>::t;
  extern __shared__ double2 lds[];
  const int S1 = kAT1 + 2 * w, S2 = kAT2 + 2 * w, K = 2 * w + 1;
  double2* tin = lds;                     // [lp][S1][S2]
  double2* tap = tin + R * S1 * S2;       // [lp][K][K], reversed
  double2* part = tap + R * K * K;        // [q - 1][kAT1 * kAT2]
  const int f = blockIdx.y / R, l = blockIdx.y - f * R;
  const int n1 = g.face_n1[f], n2 = g.face_n2[f];
  const int nt2 = (n2 + kAT2 - 1) / kAT2;
  if ((int)blockIdx.x >= ((n1 + kAT1 - 1) / kAT1) * nt2) return;  // past this face's tiles
  const int t1b = ((int)blockIdx.x / nt2) * kAT1, t2b = ((int)blockIdx.x % nt2) * kAT2;
  for (int lp = 0; lp < R; ++lp) {
    const double2* xl = xin + g.face_off[f] + (long long)lp * n1 * n2;
    for (int i = threadIdx.x; i < S1 * S2; i += kABlock) {
      const int a1 = i / S2, a2 = i - a1 * S2;
      const int j1 = t1b - w + a1, j2 = t2b - w + a2;
      tin[(lp * S1 + a1) * S2 + a2] =
          (j1 >= 0 && j1 < n1 && j2 >= 0 && j2 < n2) ? xl[(long long)j1 * n2 + j2] : make_double2(0, 0);
    }
    const double2* kl = ker + (long long)(l * R + lp) * K * K;
    for (int i = threadIdx.x; i < K * K; i += kABlock) tap[lp * K * K + i] = kl[K * K - 1 - i];
  }
  __syncthreads();
  // thread (q, o1, c): outputs (o1, 4c .. 4c + 3), tap rows d1 = q, q + kASplit, ...
  constexpr int kGroups = kAT1 * (kAT2 / 4);
  const int q = threadIdx.x / kGroups, og = threadIdx.x - q * kGroups;
  const int o1 = og / (kAT2 / 4), o2 = 4 * (og - o1 * (kAT2 / 4));
  double ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
  for (int lp = 0; lp < R; ++lp) {
    for (int d1 = q; d1 < K; d1 += kASplit) {
      const double2* irow = tin + (lp * S1 + o1 + d1) * S2 + o2;
      const double2* krow = tap + (lp * K + d1) * K;
      double2 x0 = irow[0], x1 = irow[1], x2 = irow[2];
#pragma unroll 4
      for (int d2 = 0; d2 < K; ++d2) {
        const double2 x3 = irow[d2 + 3];
        const double2 kv = krow[d2];
        ar[0] += kv.x * x0.x - kv.y * x0.y;
        ai[0] += kv.x * x0.y + kv.y * x0.x;
        ar[1] += kv.x * x1.x - kv.y * x1.y;
        ai[1] += kv.x * x1.y + kv.y * x1.x;
        ar[2] += kv.x * x2.x - kv.y * x2.y;
        ai[2] += kv.x * x2.y + kv.y * x2.x;
        ar[3] += kv.x * x3.x - kv.y * x3.y;
        ai[3] += kv.x * x3.y + kv.y * x3.x;
        x0 = x1;
        x1 = x2;
        x2 = x3;
      }
    }
  }
  if (q > 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) part[(q - 1) * kAT1 * kAT2 + o1 * kAT2 + o2 + j] = make_double2(ar[j], ai[j]);
  }
  __syncthreads();
  if (q > 0) return;
  const C* y2 = static_cast<const C*>(af.y2);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double sr = ar[j], si = ai[j];
    for (int pq = 0; pq < kASplit - 1; ++pq) {
      const double2 pv = part[pq * kAT1 * kAT2 + o1 * kAT2 + o2 + j];
      sr += pv.x;
      si += pv.y;
    }
    const int t1 = t1b + o1, t2 = t2b + o2 + j;
    if (t1 >= n1 || t2 >= n2) continue;
    const long long e = g.face_off[f] + ((long long)l * n1 + t1) * n2 + t2;
    for (int lp = 0; lp < R; ++lp) {
      const double2 av = a.m[l * R + lp];
      const long long pp = face_point(g, f, lp, t1, t2);
      const C yv = yin[pp];
      double yr = (double)yv.x, yi = (double)yv.y;
      if (y2) {
        const C zv = y2[pp];
        yr += (double)zv.x;
        yi += (double)zv.y;
      }
      sr += av.x * yr - av.y * yi;
      si += av.x * yi + av.y * yr;
    }
    double2 ov = make_double2(af.beta * sr, af.beta * si);
    if (af.base) {
      const double2 bv = af.base[e];
      ov.x += af.alpha * bv.x;
      ov.y += af.alpha * bv.y;
    }
    out[e] = ov;
  }
}

template <typename T, int R>
hipError_t shell_face_op(const abc_launch& L, const double2* x, double2* out, const typename cpx<T>::t* y,
                         const LocalBlock& a, FaceAffine af, hipStream_t st, abc_timer* tm, const char* label) {
  const Geometry& g = L.g;
  if (L.face_fft)
    return face_fft_apply<T, R>(L, x, out, nullptr, nullptr, y, a, 0.0, 3, 1, st, tm, label, af);
  if (face_affine_tiled_ok(R, L.w)) {
    int tiles = 0;
    for (int f = 0; f < 6; ++f)
      tiles = std::max(tiles, ((g.face_n1[f] + kAT1 - 1) / kAT1) * ((g.face_n2[f] + kAT2 - 1) / kAT2));
    abc_launch_kernel_lds(tm, label, face_affine_tiled_kernel<T, R>, dim3(tiles, 6 * R), dim3(kABlock),
                          face_affine_lds(R, L.w), st, x, out, y, L.face_ker, a, g, L.w, af);
  } else {
    abc_launch_kernel(tm, label, face_affine_kernel<T, R>, dim3(nblocks(g.face_off[6])), dim3(kBlock), st, x, out,
                      y, L.face_ker, a, g, L.w, af);
  }
  return hipGetLastError();
}

template <typename T, int R>
hipError_t shell_rounds_t(const abc_launch& L, const ShellScratch& W, const void* psi_v, const void* V_v,
                          const double2* f, double2* fout, void* psi_out_v, hipStream_t st, abc_timer* tm) {
  using C = typename cpx<T>::t;
  static const char* kShellLabel[4] = {"shell_1", "shell_2", "shell_3", "shell_4"};
  static const char* kFaceLabel[4] = {"shell_face_1", "shell_face_2", "shell_face_3", "shell_face_4"};
  const Geometry& g = L.g;
  const C* psi = static_cast<const C*>(psi_v);
  const T* V = static_cast<const T*>(V_v);
  C* P0 = static_cast<C*>(W.vol[0]);  // t_D, then s_D
  C* P1 = static_cast<C*>(W.vol[1]);  // v_D
  C* Q0 = static_cast<C*>(W.vol[2]);  // delta_t, then delta_s
  C* Q1 = static_cast<C*>(W.vol[3]);  // delta_v
  C* out = static_cast<C*>(psi_out_v);  // the swept state, += delta_u
  double2* F0 = W.face[0];            // t_f, then s_f
  double2* F1 = W.face[1];            // v_f
  const StencilCoef sc = make_coef(L);
  const LocalBlock a = make_local(L.a_loc);
  const double D = L.dt, a1 = L.fused_a1, b1 = L.fused_b1, a2 = L.fused_a2, b2 = L.fused_b2;
  constexpr int kAll = 1 << 30;
  auto stage = [&](int d, const C* in, int in_depth, const C* base, int base_depth, const double2* aux, C* out,
                   double alpha, double beta) {
    ShellStage<C> sp{};
    sp.box = make_shell_box(g, d);
    sp.in = in;
    sp.in_depth = in_depth;
    sp.base = base;
    sp.base_depth = base_depth;
    sp.aux = aux;
    sp.out = out;
    sp.alpha = alpha;
    sp.beta = beta;
    sp.nblk = sp.box.blk[6];
    return sp;
  };
  auto launch = [&](int k, const ShellStage<C>& sa, const ShellStage<C>& sb) {
    abc_launch_kernel(tm, kShellLabel[k], shell_stage_kernel<T, R>, dim3(sa.nblk + sb.nblk), dim3(kBlock), st, sa, sb,
                      g, V, sc);
  };
  ShellStage<C> none{};
  // round 1
  launch(0, stage(3 * R, psi, kAll, psi, kAll, nullptr, P0, a1, b1 * D),
         stage(R, nullptr, 0, nullptr, 0, f, Q0, 0.0, b1 * D));
  hipError_t e = shell_face_op<T, R>(L, f, F0, psi, a, FaceAffine{f, nullptr, a1, b1 * D}, st, tm, kFaceLabel[0]);
  if (e != hipSuccess) return e;
  // round 2
  launch(1, stage(2 * R, P0, kAll, psi, kAll, nullptr, P1, 1.0, D), stage(2 * R, Q0, R, nullptr, 0, F0, Q1, 0.0, D));
  e = shell_face_op<T, R>(L, F0, F1, P0, a, FaceAffine{f, Q0, 1.0, D}, st, tm, kFaceLabel[1]);
  if (e != hipSuccess) return e;
  // round 3
  launch(2, stage(R, P1, kAll, P1, kAll, nullptr, P0, a2, b2 * D),
         stage(3 * R, Q1, 2 * R, Q1, 2 * R, F1, Q0, a2, b2 * D));
  e = shell_face_op<T, R>(L, F1, F0, P1, a, FaceAffine{F1, Q1, a2, b2 * D}, st, tm, kFaceLabel[2]);
  if (e != hipSuccess) return e;
  // round 4
  ShellStage<C> last = stage(4 * R, Q0, 3 * R, Q1, 2 * R, F0, out, 1.0, D);
  last.accumulate = 1;
  launch(3, none, last);
  e = shell_face_op<T, R>(L, F0, fout, P0, a, FaceAffine{F1, Q0, 1.0, D}, st, tm, kFaceLabel[3]);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

template <typename T, int R, bool PER>
hipError_t step_staged_t(const abc_launch& L, const abc_scratch& S, void* psi_v, double2* aux,
                         const void* V_v, int n_steps, hipStream_t st, abc_timer* tm, void* const* keep,
                         const void* psi_in, const double2* aux_in) {
  static const char* kStageLabel[5] = {"", "stage_1", "stage_2", "stage_3", "stage_4"};
  static const char* kBoundLabel[5] = {"", "boundary_1", "boundary_2", "boundary_3", "boundary_4"};
  using C = typename cpx<T>::t;
  const Geometry& g = L.g;
  C* psi = static_cast<C*>(psi_v);
  const T* V = static_cast<const T*>(V_v);
  C* y[2] = {static_cast<C*>(S.y[0]), static_cast<C*>(S.y[1])};
  C* acc = static_cast<C*>(S.acc);
  const StencilCoef sc = make_coef(L);
  const LocalBlock a = make_local(L.a_loc);
  const long long nel = g.npts * g.batch;
  const long long nface = g.face_off[6];
  // one orbital, zero outside the box: the tiled sweep
  const bool tiled = !PER && g.batch == 1 && R >= kTiledMinR;
  const TileGrid tg = make_tile_grid(g, TileShape<R, kTileJ>::TY, tile_planes(R));
  const unsigned ntile = (unsigned)(tg.ntx * tg.nty * tg.ntz);
  const bool zeroth = L.order == ABC_ZEROTH;
  // boundary variables with their own recurrence: f (first), f and g (second)
  const bool rec = L.order == ABC_FIRST || L.order == ABC_SECOND;
  const bool box = L.form == ABC_FORM_BOX;
  for (int s = 0; s < n_steps; ++s) {
    // this step's input state (the first step may read it from elsewhere)
    const C* pin = (s == 0 && psi_in) ? static_cast<const C*>(psi_in) : psi;
    const T* Vuse = V;
    if (L.meanfield == ABC_MF_SKYRME) {
      const hipError_t e = skyrme_veff(*L.pot, pin, false, g.batch, sizeof(T) == 4, V, S.veff, L.t0, L.t3, st, tm);
      if (e != hipSuccess) return e;
      Vuse = static_cast<const T*>(S.veff);
    } else if (L.meanfield) {
      abc_launch_kernel(tm, "meanfield", meanfield_kernel<T>, dim3(nblocks(g.npts)), dim3(kBlock), st, pin, V,
                        static_cast<T*>(S.veff), g.npts, g.batch, T(L.t0), T(L.t3));
      Vuse = static_cast<const T*>(S.veff);
    }
    const C* ycur = pin;
    const double2* gcur = (s == 0 && aux_in) ? aux_in : aux;  // g_0 = f
    for (int k = 1; k <= 4; ++k) {
      const double coef = L.dt / k;
      const int mode = k == 1 ? 0 : (k == 4 ? 2 : 1);
      const double2* fsrc = nullptr;
      const double2* bsrc = nullptr;
      // the boundary-variable stage runs in the stage's launch (its output)
      bool merged = false;
      double2* merged_gnext = nullptr;
      if (rec || zeroth) {
        double2* gnext = (k == 4) ? nullptr : S.g[(k - 1) & 1];
        if (box && g.batch > 1) {
          // one complex GEMM over the orbitals on the matrix cores: T =
          // [B | A] [g; E y] (first), the 2n rows of the second order, or
          // M E y (zeroth); the operator is read once for all orbitals
          const int n = L.n_gamma, nb = g.batch;
          const int na = abc::box_aux_rows(L.order, n), rows = abc::box_rows(L.order, n);
          const int ld = abc::box_cols(L.order, n);
          const long long cnt = (long long)rows * nb, ng = (long long)n * nb;
          abc_launch_kernel(tm, kBoundLabel[k], box_gather_kernel<T>, dim3(nblocks(ng)), dim3(kBlock), st,
                            (const C*)ycur, L.gamma_lin, n, nb, S.bwork[0]);
          double2* tout = rec ? S.bwork[1] : S.src;
          const hipError_t ge = box_gemm(tm, L.box_mat, rows, ld, na, rec ? gcur : nullptr,
                                         (const double2*)S.bwork[0], nb, tout, S.bpart, st);
          if (ge != hipSuccess) return ge;
          if (rec)
            abc_launch_kernel(tm, "box_epilogue", box_epilogue_kernel, dim3(nblocks(cnt)), dim3(kBlock), st,
                              (const double2*)tout, gcur, gnext, S.facc, aux, cnt, coef, mode);
        } else if (box && g.batch == 1 && L.box_r > 0 && L.order == ABC_SECOND && S.bpack) {
          // second order in the DtN maps' dominant subspace
          const hipError_t e = second_reduced_stage<T>(L, S, (const C*)ycur, gcur, gnext, aux, coef, mode, st, tm,
                                                       kBoundLabel[k]);
          if (e != hipSuccess) return e;
        } else if (box && g.batch == 1 && S.bwork[0] && abc::box_rows(L.order, L.n_gamma) >= kBoxRowsMin) {
          // one orbital, large operator: gather E y, then kBoxRows rows per
          // workgroup (below kBoxRowsMin rows the extra launch and the fewer
          // workgroups cost more than the shared vector loads save)
          const int n = L.n_gamma, rows = abc::box_rows(L.order, n);
          abc_launch_kernel(tm, kBoundLabel[k], box_gather_kernel<T>, dim3(nblocks(n)), dim3(kBlock), st,
                            (const C*)ycur, L.gamma_lin, n, 1, S.bwork[0]);
          abc_launch_kernel(tm, kBoundLabel[k], box_gemv_rows_kernel, dim3((rows + kBoxRows - 1) / kBoxRows),
                            dim3(kBlock), st, (const double2*)L.box_mat, rows, abc::box_aux_rows(L.order, n),
                            abc::box_cols(L.order, n), L.order == ABC_SECOND ? n : 0, gcur,
                            (const double2*)S.bwork[0], rec ? gnext : S.src, S.facc, aux, coef, mode);
        } else if (box) {
          const int n = L.n_gamma;
          dim3 grid(abc::box_rows(L.order, n), g.batch);
          abc_launch_kernel(tm, kBoundLabel[k], box_gemv_kernel<T>, grid, dim3(kBlock), st, L.box_mat,
                            abc::box_aux_rows(L.order, n), abc::box_cols(L.order, n),
                            L.order == ABC_SECOND ? n : 0, gcur, ycur, L.gamma_lin,
                            rec ? gnext : S.src, S.facc, aux, g.batch, coef, mode);
        } else if (L.face_fft) {
          const hipError_t e = face_fft_apply<T, R>(L, gcur, rec ? gnext : S.src, S.facc, aux, ycur, a, coef, mode,
                                                    rec ? 1 : 0, st, tm, kBoundLabel[k]);
          if (e != hipSuccess) return e;
        } else if (rec && L.w == 0) {
          // local operator: launched with the stage below (with a window the
          // face work is heavy enough that the combined launch is slower
          // than two: 128^3, w = 8, 409 against 333 us per step)
          merged = true;
          merged_gnext = gnext;
        } else if (face_tiled_ok(R, L.w, g.batch)) {
          int tiles = 0;
          for (int f = 0; f < 6; ++f)
            tiles = std::max(tiles, ((g.face_n1[f] + kFT - 1) / kFT) * ((g.face_n2[f] + kFT - 1) / kFT));
          abc_launch_kernel(tm, kBoundLabel[k], face_tiled_kernel<T, R>, dim3(tiles, 6 * R), dim3(kFBlock), st, gcur,
                            rec ? gnext : S.src, S.facc, aux, ycur, L.face_ker, a, g, L.w, coef, mode,
                            rec ? 1 : 0);
        } else {
          abc_launch_kernel(tm, kBoundLabel[k], face_kernel<T, R>, dim3(nblocks(nface)), dim3(kBlock), st, gcur,
                            rec ? gnext : S.src, S.facc, aux, ycur, L.face_ker, a, g, L.w, coef, mode,
                            rec ? 1 : 0);
        }
        const double2* s_for_stage = rec ? gcur : S.src;
        if (box) bsrc = s_for_stage; else fsrc = s_for_stage;
        if (rec) gcur = gnext;
      }
      C* yout = (k == 4) ? nullptr : (keep ? static_cast<C*>(keep[k - 1]) : y[(k - 1) & 1]);
      // the stage sweep's own mode (the face work keeps `mode`): stage 2
      // starts the running sum from the step's input state, read through
      // `state`; stage 4 finishes it into the new state
      const int smode = k == 2 ? 1 : (k == 4 ? 2 : 0);
      C* state = k == 2 ? const_cast<C*>(pin) : psi;
      if (merged && tiled) {
        abc_launch_kernel(tm, kStageLabel[k], stage_face_tiled_kernel<T, R, kTileJ>,
                          dim3(ntile + (unsigned)((nface + kTiledBlock(R) - 1) / kTiledBlock(R))),
                          dim3(kTiledBlock(R)), st, tg, ycur, yout, acc, state, Vuse, fsrc, L.point_gamma, sc, fsrc,
                          merged_gnext, S.facc, aux, L.face_ker, a, g, L.w, coef, smode, mode, ntile);
      } else if (merged) {
        const unsigned nsb = (unsigned)nblocks(nel);
        abc_launch_kernel(tm, kStageLabel[k], stage_face_kernel<T, R, PER>, dim3(nsb + nblocks(nface)), dim3(kBlock),
                          st, ycur, yout, acc, state, Vuse, fsrc, L.point_gamma, sc, fsrc, merged_gnext, S.facc, aux,
                          L.face_ker, a, g, L.w, coef, smode, mode, nsb);
      } else if (tiled) {
        abc_launch_kernel(tm, kStageLabel[k], stage_tiled_kernel<T, R, kTileJ>, dim3(ntile), dim3(kTiledBlock(R)), st, tg,
                          ycur, yout, acc, state, Vuse, fsrc, bsrc, L.point_gamma, g, sc, coef, smode);
      } else {
        abc_launch_kernel(tm, kStageLabel[k], stage_kernel<T, R, PER>, dim3(nblocks(nel)), dim3(kBlock), st, ycur,
                          yout, acc, state, Vuse, fsrc, bsrc, L.point_gamma, g, sc, coef, smode);
      }
      ycur = yout;
    }
    if (tm) tm->end_step();
  }
  return hipGetLastError();
}

template <typename T, int R, bool PER>
hipError_t diag_t(const abc_launch& L, double* red, const void* psi, const double2* aux, const void* V,
                  double* out, hipStream_t st) {
  using C = typename cpx<T>::t;
  const Geometry& g = L.g;
  const StencilCoef sc = make_coef(L);
  dim3 grid(kRedBlocks, g.batch);
  diag_points_kernel<T, R, PER><<<grid, kBlock, 0, st>>>(static_cast<const C*>(psi), static_cast<const T*>(V), g, sc,
                                                         L.meanfield, L.t0, L.t3, red);
  const int has_aux = (L.order == ABC_FIRST && aux) ? 1 : 0;
  if (has_aux) {
    dim3 ga(kAuxBlocks, g.batch);
    if (L.form == ABC_FORM_BOX) {
      diag_box_aux_kernel<<<ga, kBlock, 0, st>>>(aux, L.box_q, L.n_gamma, g.batch, red);
    } else {
      long long lines = 0;
      for (int f = 0; f < 6; ++f) lines += (long long)g.face_n1[f] * g.face_n2[f];
      diag_aux_kernel<R><<<ga, kBlock, 0, st>>>(aux, g, make_local(L.q_loc), lines, red);
    }
  }
  diag_finish_kernel<<<(g.batch + 63) / 64, 64, 0, st>>>(red, g.batch, L.h * L.h * L.h, has_aux, out);
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_step(const abc_launch& L, const abc_scratch& S, void* psi, double2* aux, const void* V,
                         int n, hipStream_t st, abc_timer* tm, void* const* keep, const void* pin,
                         const double2* ain) {
  const bool per = L.periodic != 0;
  switch (L.g.R) {
    case 1: return per ? step_staged_t<T, 1, true>(L, S, psi, aux, V, n, st, tm, keep, pin, ain) : step_staged_t<T, 1, false>(L, S, psi, aux, V, n, st, tm, keep, pin, ain);
    case 2: return per ? step_staged_t<T, 2, true>(L, S, psi, aux, V, n, st, tm, keep, pin, ain) : step_staged_t<T, 2, false>(L, S, psi, aux, V, n, st, tm, keep, pin, ain);
    case 3: return per ? step_staged_t<T, 3, true>(L, S, psi, aux, V, n, st, tm, keep, pin, ain) : step_staged_t<T, 3, false>(L, S, psi, aux, V, n, st, tm, keep, pin, ain);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t dispatch_diag(const abc_launch& L, double* red, const void* psi, const double2* aux,
                         const void* V, double* out, hipStream_t st) {
  const bool per = L.periodic != 0;
  switch (L.g.R) {
    case 1: return per ? diag_t<T, 1, true>(L, red, psi, aux, V, out, st) : diag_t<T, 1, false>(L, red, psi, aux, V, out, st);
    case 2: return per ? diag_t<T, 2, true>(L, red, psi, aux, V, out, st) : diag_t<T, 2, false>(L, red, psi, aux, V, out, st);
    case 3: return per ? diag_t<T, 3, true>(L, red, psi, aux, V, out, st) : diag_t<T, 3, false>(L, red, psi, aux, V, out, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace

size_t box_gemm_part_elems(size_t result_elems) { return (size_t)kGemmMaxKs * result_elems; }

hipError_t launch_step_staged(const abc_launch& L, const abc_scratch& S, void* psi, double2* aux, const void* V,
                              int n_steps, hipStream_t st, abc_timer* tm, void* const* keep, const void* psi_in,
                              const double2* aux_in) {
  if (L.dtype == ABC_C64) return dispatch_step<float>(L, S, psi, aux, V, n_steps, st, tm, keep, psi_in, aux_in);
  return dispatch_step<double>(L, S, psi, aux, V, n_steps, st, tm, keep, psi_in, aux_in);
}

hipError_t launch_diagnostics(const abc_launch& L, const abc_scratch& S, const void* psi, const double2* aux,
                              const void* V, double* out, hipStream_t st, double* red) {
  if (!red) red = S.red;
  if (L.dtype == ABC_C64) return dispatch_diag<float>(L, red, psi, aux, V, out, st);
  return dispatch_diag<double>(L, red, psi, aux, V, out, st);
}

size_t diag_partial_doubles(int batch) { return (size_t)batch * (kRedBlocks + kAuxBlocks) * 4; }

// Monitor record check (one block).  rec = [step, the 3 B + 1 diagnostics]:
// stores the step count, raises ABC_FLAG_NONFINITE if a diagnostic is NaN or
// infinite and, with check_w, ABC_FLAG_W_INCREASE if an orbital's W exceeds
// its previous record by more than tol of that value (the zeroth- and
// first-order theorems of Sec. 3 make W non-increasing); the new W values
// then become the previous ones.
__global__ void __launch_bounds__(256) monitor_check_kernel(double* __restrict__ rec, int B, double step,
                                                            double* __restrict__ prevW, int have_prev, int check_w,
                                                            double tol, unsigned* __restrict__ flags) {
  const int t = threadIdx.x;
  if (t == 0) rec[0] = step;
  const double* d = rec + 1;
  unsigned f = 0;
  for (int i = t; i < 3 * B + 1; i += blockDim.x)
    if (!isfinite(d[i])) f |= ABC_FLAG_NONFINITE;
  for (int j = t; j < B; j += blockDim.x) {
    const double w = d[B + j];
    if (check_w && have_prev && w - prevW[j] > tol * fabs(prevW[j])) f |= ABC_FLAG_W_INCREASE;
    prevW[j] = w;
  }
  if (f) atomicOr(flags, f);
}

hipError_t launch_monitor_check(double* rec, int batch, long long step, double* prevW, bool have_prev, bool check_w,
                                double tol, unsigned* flags, hipStream_t st) {
  monitor_check_kernel<<<1, 256, 0, st>>>(rec, batch, (double)step, prevW, have_prev ? 1 : 0, check_w ? 1 : 0, tol,
                                          flags);
  return hipGetLastError();
}

// FFT plan of the exact face sections: padded sizes per face pair, work
// slabs, twiddle tables, and the kernel spectra (the padded R x R kernel
// layers transformed on the device)
abc_status face_fft_setup(const Geometry& g, int R, int w, const std::vector<abc::cd>& kernel, FaceFFT& ff,
                          std::vector<void*>* allocs, size_t* bytes, std::string& err) {
  const int K = 2 * w + 1, B = g.batch;
  long long woff = 0, soff = 0;
  std::vector<double2> tw;
  for (int q = 0; q < 3; ++q) {
    const int n1 = g.face_n1[2 * q], n2 = g.face_n2[2 * q];
    if (w < n1 - 1 || w < n2 - 1) { err = "the FFT face path needs the exact section (window >= n - 1)"; return ABC_EINVAL; }
    int P1 = 2, P2 = 2;
    while (P1 < 2 * n1 - 1) P1 *= 2;
    while (P2 < 2 * n2 - 1) P2 *= 2;
    if (P1 > 4096 || P2 > 4096) { err = "face too large for the FFT face path"; return ABC_ENOTSUP; }
    ff.P1[q] = P1;
    ff.P2[q] = P2;
    ff.S[q] = 2 * R * B;
    ff.lg1[q] = ilog2(P1);
    ff.lg2[q] = ilog2(P2);
    // row passes: kBlock points per workgroup (one 256-point line: 180.5
    // against 184 us per step at 128^3 with two); column passes: two lines
    // (one, four, eight or sixteen were slower: 196, 188, 203, 251 us)
    ff.twr[q] = std::min(ff.S[q] * n1, std::max(1, kBlock / P2));
    int twc = fft_lines_per_group(P1, P2, 2);
    while (twc > 1 && R * twc * P1 > 4096) twc >>= 1;
    if (R * twc * P1 > 4096) { err = "face too large for the FFT face path at this stencil radius"; return ABC_ENOTSUP; }
    ff.twc[q] = twc;
    // twiddles in LDS behind the lines where the 64 KB allow
    ff.stwr[q] = ff.twr[q] * P2 + P2 / 2 <= 4096;
    ff.stwc[q] = R * twc * P1 + P1 / 2 <= 4096;
    ff.woff[q] = woff;
    woff += (long long)ff.S[q] * P1 * P2;
    ff.soff[q] = soff;
    soff += (long long)R * R * P1 * P2;
    const int Ls[4] = {P2, P2, P1, P1};
    const double sg[4] = {-1.0, 1.0, -1.0, 1.0};
    for (int j = 0; j < 4; ++j) {
      ff.twoff[q][j] = (long long)tw.size();
      for (int k = 0; k < Ls[j] / 2; ++k)
        tw.push_back(make_double2(std::cos(2 * M_PI * k / Ls[j]), sg[j] * std::sin(2 * M_PI * k / Ls[j])));
    }
  }
  ff.woff[3] = woff;
  ff.soff[3] = soff;
  std::vector<double2> spec((size_t)soff, make_double2(0.0, 0.0));
  for (int q = 0; q < 3; ++q) {
    const int n1 = g.face_n1[2 * q], n2 = g.face_n2[2 * q], P1 = ff.P1[q], P2 = ff.P2[q];
    for (int l = 0; l < R; ++l)
      for (int lp = 0; lp < R; ++lp) {
        double2* dst = spec.data() + ff.soff[q] + (long long)(l * R + lp) * P1 * P2;
        for (int p1 = -(n1 - 1); p1 <= n1 - 1; ++p1)
          for (int p2 = -(n2 - 1); p2 <= n2 - 1; ++p2) {
            const abc::cd v = kernel[((size_t)(l * R + lp) * K + (p1 + w)) * K + (p2 + w)];
            dst[(size_t)((p1 + P1) % P1) * P2 + (p2 + P2) % P2] = make_double2(v.real(), v.imag());
          }
      }
  }
  void *pw = nullptr, *pz = nullptr, *ps = nullptr, *pt = nullptr;
  const size_t wb = (size_t)woff * sizeof(double2), sb = (size_t)soff * sizeof(double2), tb = tw.size() * sizeof(double2);
  auto dalloc = [&](void** ptr, size_t nbytes) {
    if (hipMalloc(ptr, nbytes) != hipSuccess) return false;
    allocs->push_back(*ptr);
    *bytes += nbytes;
    return true;
  };
  if (!dalloc(&pw, wb) || !dalloc(&pz, wb) || !dalloc(&ps, sb) || !dalloc(&pt, tb)) {
    err = "device allocation for the FFT face path failed";
    return ABC_ENOMEM;
  }
  ff.W = static_cast<double2*>(pw);
  ff.Z = static_cast<double2*>(pz);
  ff.spec = static_cast<double2*>(ps);
  ff.tw = static_cast<double2*>(pt);
  if (hipMemcpy(ff.spec, spec.data(), sb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(ff.tw, tw.data(), tb, hipMemcpyHostToDevice) != hipSuccess) {
    err = "hipMemcpy failed";
    return ABC_EDEVICE;
  }
  for (int q = 0; q < 3; ++q)
    if (fft2_slabs(ff.spec + ff.soff[q], ff.P1[q], ff.P2[q], R * R, ff.tw + ff.twoff[q][0], ff.tw + ff.twoff[q][2],
                   nullptr) != hipSuccess) {
      err = "kernel spectra transform failed";
      return ABC_EDEVICE;
    }
  if (hipDeviceSynchronize() != hipSuccess) { err = "kernel spectra transform failed"; return ABC_EDEVICE; }
  return ABC_OK;
}

hipError_t launch_shell_rounds(const abc_launch& L, const ShellScratch& W, const void* psi, const void* V,
                               const double2* f, double2* fout, void* psi_out, hipStream_t st, abc_timer* tm) {
  if (L.g.R != 1 || L.g.batch != 1) return hipErrorInvalidValue;
  if (L.dtype == ABC_C64) return shell_rounds_t<float, 1>(L, W, psi, V, f, fout, psi_out, st, tm);
  return shell_rounds_t<double, 1>(L, W, psi, V, f, fout, psi_out, st, tm);
}
