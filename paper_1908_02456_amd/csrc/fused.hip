// Fused Taylor-4 step: all four stages of z_k = (dt/k) L z_{k-1} and the
// accumulation psi' = z_0 + ... + z_4 (Sec. 4 Taylor propagator) in one
// sweep, with the boundary terms of the face-form conditions (Sec. 3) when
// the face operators are local (window 0).
//
// Layout of the sweep (R = 1):
//   * a workgroup owns an output tile of all x (<= 128), 8 rows in y and 8
//     planes in z; it loads 4-deep halos in y and z (one per stage);
//   * one wavefront per y row (16 rows = 8 output + 2 x 4 halo), each lane
//     holding two consecutive x columns, so x needs no halo;
//   * the workgroup marches z: when plane zi is loaded, stage k works on
//     plane zi - k.  Each stage keeps the plane below and the centre plane of
//     its input in registers (the plane above is the previous stage's fresh
//     output) and publishes its centre plane in LDS for the x/y neighbours;
//   * the first-order auxiliary recurrence g_k = (dt/k)(b g_{k-1} + a y_{k-1})
//     is carried per face point along the same pipeline (z faces in
//     registers, x and y faces in LDS slots);
//   * tiles are mapped so that consecutive tiles share an XCD (and its L2),
//     which keeps the halo re-reads on chip.
// psi and the auxiliary slab are read from one buffer and written to another
// (neighbouring tiles read halos that this tile overwrites).
#include <hip/hip_runtime.h>

#include "fused.h"

namespace {

constexpr int kTY = 8;
constexpr int kTZ = 8;
constexpr int kHalo = 4;
constexpr int kRows = kTY + 2 * kHalo;  // 16 wavefronts
constexpr int kCols = 128;
constexpr int kThreads = 64 * kRows;
constexpr int kIters = kTZ + 2 * kHalo;

template <typename T> struct cpx;
template <> struct cpx<double> { using t = double2; };
template <> struct cpx<float> { using t = float2; };

struct FusedArgs {
  int nx, ny, nz;
  int nty, ntiles, tiles_per_xcd;
  double diag, off;
  double coef[5];
  double2 m0, b0, a0;
  int face_off[7];
  int has_V;
};

template <typename C>
__device__ __forceinline__ C czero() {
  C z;
  z.x = 0;
  z.y = 0;
  return z;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ORDER: 0 = no condition (zero outside), 2 = zeroth order, 3 = first order.
//
// The four stages are evaluated in Horner form, which is the same
// polynomial sum_{k<=4} (dt L)^k / k! with a different rounding order:
//   u3 = z0 + (dt/4) L z0,  u2 = z0 + (dt/3) L u3,  u1 = z0 + (dt/2) L u2,
//   z' = z0 + dt L u1,       z0 = (psi, f).
// Nothing has to be accumulated across planes: stage k only needs the
// initial state at its own plane (registers for stages 1-2, a cached
// re-read for stages 3-4).
template <typename T, int ORDER>
__global__ void __launch_bounds__(kThreads) fused_step_kernel(
    const typename cpx<T>::t* __restrict__ pin, typename cpx<T>::t* __restrict__ pout, const T* __restrict__ V,
    const double2* __restrict__ fin, double2* __restrict__ fout, FusedArgs a) {
  using C = typename cpx<T>::t;
  __shared__ C plane[4][kRows][kCols];
  constexpr int GX = ORDER == 3 ? kRows : 1;
  constexpr int GY = ORDER == 3 ? kCols : 1;
  __shared__ double2 gx[2][3][2][GX];  // x-face aux stages [side][stage-1][parity][row]
  __shared__ double2 gy[2][3][2][GY];  // y-face aux stages [side][stage-1][parity][x]

  const int lane = threadIdx.x & 63;
  const int r = threadIdx.x >> 6;
  int tile = blockIdx.x;
  if (a.tiles_per_xcd) tile = (blockIdx.x & 7) * a.tiles_per_xcd + (blockIdx.x >> 3);
  const int ty = tile % a.nty, tz = tile / a.nty;
  const int y0 = ty * kTY, z0 = tz * kTZ;
  const int y = y0 - kHalo + r;
  const bool row_in = y >= 0 && y < a.ny;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int sz = nx * ny;
  const int ybase = y * nx;
  const bool own_row = r >= kHalo && r < kHalo + kTY && row_in;

  for (int i = threadIdx.x; i < 4 * kRows * kCols; i += kThreads) (&plane[0][0][0])[i] = czero<C>();
  __syncthreads();

  // Yc[j] / Yb[j]: stage-j output at the centre / below plane of stage j+1
  C Yc[4][2], Yb[4][2];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int c = 0; c < 2; ++c) Yc[j][c] = Yb[j][c] = czero<C>();
  double2 gz[2] = {make_double2(0, 0), make_double2(0, 0)};

  const T diag = T(a.diag), off = T(a.off);

  for (int it = 0; it < kIters; ++it) {
    const int zi = z0 - kHalo + it;
    C nw[5][2];
    const bool load_ok = row_in && zi >= 0 && zi < nz;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int x = 2 * lane + c;
      nw[0][c] = (load_ok && x < nx) ? pin[zi * sz + ybase + x] : czero<C>();
    }
#pragma unroll
    for (int k = 1; k <= 4; ++k) {
      const int zk = zi - k;
      const bool active = r >= k && r < kRows - k && it >= 2 * k && row_in && zk >= 0 && zk < nz;
      if (!active) {
        nw[k][0] = nw[k][1] = czero<C>();
        continue;
      }
      const T cf = T(a.coef[5 - k]);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int x = 2 * lane + c;
        if (x >= nx) {
          nw[k][c] = czero<C>();
          continue;
        }
        const C cen = Yc[k - 1][c], bel = Yb[k - 1][c], abv = nw[k - 1][c];
        const C ym = plane[k - 1][r - 1][x];
        const C yp = plane[k - 1][r + 1][x];
        C xm, xp;
        if (c == 0) {
          xm = x > 0 ? plane[k - 1][r][x - 1] : czero<C>();
          xp = Yc[k - 1][1];
        } else {
          xm = Yc[k - 1][0];
          xp = (x + 1 < kCols) ? plane[k - 1][r][x + 1] : czero<C>();
        }
        // initial state at this plane: centre of stage 1, below of stage 1,
        // re-read for stages 3 and 4
        C z0v;
        if (k == 1) z0v = Yc[0][c];
        else if (k == 2) z0v = Yb[0][c];
        else z0v = pin[zk * sz + ybase + x];
        T hr = diag * cen.x + off * (bel.x + abv.x + ym.x + yp.x + xm.x + xp.x);
        T hi = diag * cen.y + off * (bel.y + abv.y + ym.y + yp.y + xm.y + xp.y);
        if (a.has_V) {
          const T v = V[zk * sz + ybase + x];
          hr += v * cen.x;
          hi += v * cen.y;
        }
        if (ORDER == 2) {
          const int nf = (x == 0) + (x == nx - 1) + (y == 0) + (y == ny - 1) + (zk == 0) + (zk == nz - 1);
          if (nf) {
            const double2 s = cmul(a.m0, make_double2((double)cen.x, (double)cen.y));
            hr += T(nf * s.x);
            hi += T(nf * s.y);
          }
        }
        if (ORDER == 3) {
          // aux stage v_k = f + c_k (b v_{k-1} + a u_{k-1}) per face point;
          // the psi stage sees the sum of v_{k-1} over the faces at the point
          const bool own = own_row && zk >= z0 && zk < z0 + kTZ && k == 4;
          const double2 yc = make_double2((double)cen.x, (double)cen.y);
          const double cfd = a.coef[5 - k];
          double sr = 0, si = 0;
          auto aux_stage = [&](int idx, double2 vp) {
            const double2 f0 = fin[idx];
            const double2 t1 = cmul(a.b0, vp), t2 = cmul(a.a0, yc);
            sr += vp.x;
            si += vp.y;
            return make_double2(f0.x + cfd * (t1.x + t2.x), f0.y + cfd * (t1.y + t2.y));
          };
          if (x == 0 || x == nx - 1) {  // x faces: (t_slow, t_fast) = (z, y)
            const int side = x == 0 ? 0 : 1;
            const int idx = a.face_off[side] + zk * ny + y;
            const double2 vp = k == 1 ? fin[idx] : gx[side][k - 2][(it - 1) & 1][r];
            const double2 vk = aux_stage(idx, vp);
            if (k <= 3) gx[side][k - 1][it & 1][r] = vk;
            if (own) fout[idx] = vk;
          }
          if (y == 0 || y == ny - 1) {  // y faces: (z, x)
            const int side = y == 0 ? 0 : 1;
            const int idx = a.face_off[2 + side] + zk * nx + x;
            const double2 vp = k == 1 ? fin[idx] : gy[side][k - 2][(it - 1) & 1][x];
            const double2 vk = aux_stage(idx, vp);
            if (k <= 3) gy[side][k - 1][it & 1][x] = vk;
            if (own) fout[idx] = vk;
          }
          if (zk == 0 || zk == nz - 1) {  // z faces: (y, x); one stage per iteration
            const int side = zk == 0 ? 0 : 1;
            const int idx = a.face_off[4 + side] + ybase + x;
            const double2 vp = k == 1 ? fin[idx] : gz[c];
            const double2 vk = aux_stage(idx, vp);
            gz[c] = vk;
            if (own) fout[idx] = vk;
          }
          hr += T(sr);
          hi += T(si);
        }
        C o;
        o.x = z0v.x + cf * hi;
        o.y = z0v.y - cf * hr;
        nw[k][c] = o;
      }
    }
    // stage 4 output is the new state at plane zi - 4
    const int z4 = zi - 4;
    const bool own_out = own_row && it >= 2 * kHalo && z4 < nz;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int x = 2 * lane + c;
      if (own_out && x < nx) pout[z4 * sz + ybase + x] = nw[4][c];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        Yb[j][c] = Yc[j][c];
        Yc[j][c] = nw[j][c];
      }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int c = 0; c < 2; ++c) plane[j][r][2 * lane + c] = Yc[j][c];
    __syncthreads();
  }
}

FusedArgs make_args(const abc_launch& L) {
  FusedArgs a{};
  a.nx = L.g.nx;
  a.ny = L.g.ny;
  a.nz = L.g.nz;
  a.nty = (a.ny + kTY - 1) / kTY;
  const int ntz = (a.nz + kTZ - 1) / kTZ;
  a.ntiles = a.nty * ntz;
  a.tiles_per_xcd = (a.ntiles % 8 == 0) ? a.ntiles / 8 : 0;
  const double s = 1.0 / (2.0 * L.h * L.h);
  a.diag = -3.0 * L.c[0] * s;
  a.off = -L.c[1] * s;
  for (int k = 1; k <= 4; ++k) a.coef[k] = L.dt / k;
  for (int f = 0; f < 7; ++f) a.face_off[f] = (int)L.g.face_off[f];
  return a;
}

}  // namespace

bool fused_supported(const abc_params& p, std::string* why) {
  auto no = [&](const char* m) {
    if (why) *why = m;
    return false;
  };
  if (p.radius != 1) return no("radius 1 only");
  if (p.batch != 1) return no("batch 1 only");
  if (p.meanfield != ABC_MF_NONE) return no("no mean field");
  if (p.order == ABC_PERIODIC) return no("periodic boxes use the staged path");
  if ((p.order == ABC_ZEROTH || p.order == ABC_FIRST) && (p.form != ABC_FORM_FACES || p.window != 0))
    return no("local (window 0) face operators only");
  if (p.nx > kCols) return no("nx <= 128");
  if (p.nz < 5 || p.ny < 3) return no("ny >= 3 and nz >= 5");
  if ((long long)p.nx * p.ny * p.nz >= (1LL << 31)) return no("grid below 2^31 points");
  return true;
}

abc_status fused_prepare(const abc_params& p, abc_launch& L, std::vector<void*>* allocs, size_t* bytes,
                         std::string& err) {
  (void)p;
  (void)allocs;
  (void)bytes;
  (void)err;
  (void)L;
  return ABC_OK;
}

namespace {

template <typename T>
hipError_t step_t(const abc_launch& L, const abc_scratch& S, void* psi_v, double2* aux, const void* V_v, int n,
                  hipStream_t st) {
  using C = typename cpx<T>::t;
  FusedArgs a = make_args(L);
  a.m0 = L.fused_m0;
  a.b0 = L.fused_b0;
  a.a0 = L.a_loc[0];
  a.has_V = V_v != nullptr;
  C* user = static_cast<C*>(psi_v);
  C* scr = static_cast<C*>(S.y[0]);
  double2* fuser = aux;
  double2* fscr = S.facc;
  const bool first = L.order == ABC_FIRST;
  const size_t pbytes = (size_t)L.g.npts * sizeof(C);
  const size_t fbytes = (size_t)L.g.face_off[6] * sizeof(double2);
  // arrange the ping-pong so that the last step writes the caller's buffers
  C* src = user;
  C* dst = scr;
  double2* fsrc = fuser;
  double2* fdst = fscr;
  if (n & 1) {
    hipError_t e = hipMemcpyAsync(scr, user, pbytes, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    if (first) {
      e = hipMemcpyAsync(fscr, fuser, fbytes, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return e;
    }
    src = scr;
    dst = user;
    fsrc = fscr;
    fdst = fuser;
  }
  const T* V = static_cast<const T*>(V_v);
  for (int s = 0; s < n; ++s) {
    switch (L.order) {
      case ABC_ZEROTH:
        fused_step_kernel<T, 2><<<a.ntiles, kThreads, 0, st>>>(src, dst, V, nullptr, nullptr, a);
        break;
      case ABC_FIRST:
        fused_step_kernel<T, 3><<<a.ntiles, kThreads, 0, st>>>(src, dst, V, fsrc, fdst, a);
        break;
      default:
        fused_step_kernel<T, 0><<<a.ntiles, kThreads, 0, st>>>(src, dst, V, nullptr, nullptr, a);
        break;
    }
    std::swap(src, dst);
    std::swap(fsrc, fdst);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step_fused(const abc_launch& L, const abc_scratch& S, void* psi, double2* aux, const void* V,
                             int n_steps, hipStream_t st) {
  if (L.dtype == ABC_C64) return step_t<float>(L, S, psi, aux, V, n_steps, st);
  return step_t<double>(L, S, psi, aux, V, n_steps, st);
}
