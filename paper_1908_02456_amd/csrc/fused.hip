// Fused Taylor-4 step kernels (Sec. 4 Taylor propagator applied to the
// dynamics of Sec. 3), for R = 1 and local (window 0) face operators.
//
// The step U = sum_{k<=4} (dt L)^k / k! is evaluated in Horner form, the same
// polynomial with a different rounding order:
//   u3 = z0 + (dt/4) L z0,  u2 = z0 + (dt/3) L u3,  u1 = z0 + (dt/2) L u2,
//   z' = z0 + dt L u1,       z0 = (psi, f).
//
// Sweep layout:
//   * a workgroup owns an output tile of one x chunk (the whole row up to 128
//     columns), TY rows in y and TZ planes in z, and loads one halo row/plane
//     per fused stage on each side;
//   * one wavefront per y row, two consecutive x columns per lane; rows are
//     published in LDS as [column parity][1 + lane] with a zero guard cell at
//     each end (conflict-free, branch-free x neighbours);
//   * the workgroup marches z: when plane zi is loaded, stage k works on plane
//     zi - k with its input's below/centre planes in registers, the plane above
//     being the previous stage's fresh output; the initial state needed by the
//     Horner stages rides along in a register delay line;
//   * tiles are numbered so that consecutive tiles share an XCD and its L2.
// fused2_kernel runs two of the four stages per launch (two launches per step,
// two-deep halos) and also carries the zeroth- and first-order conditions.
// The first-order auxiliary stages are formed at face points only: on the x
// faces and the y-face row by the two halo waves (which do no stencil work),
// through small LDS rings; on the z-face plane by the row waves from
// registers.  The face sources enter the stage outputs of the face points
// (whole rows on y and z faces, one column at each end of a row on x faces).
// The state is read from one buffer and written to another, since
// neighbouring tiles read halos that a tile overwrites.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <type_traits>
#include <utility>

#include "fused.h"

namespace {

constexpr int kCols = 128;

template <typename T> struct cpx;
template <> struct cpx<double> { using t = double2; };
template <> struct cpx<float> { using t = float2; };

struct FusedArgs {
  int nx, ny, nz;
  int ntx, xw;  // x chunks and output columns per chunk (two-stage kernel)
  int nty, ntiles, tiles_per_xcd;
  double diag, off;
  double coef[5];
  double sa1, sa2;  // one-pass sweep: base scales of stages 1 and 3 (factored form)
  double2 m0, b0, a0;
  int face_off[7];
  int has_V;
  long long bstride, fstride;  // one-pass sweep over orbitals: elements between orbitals' psi / aux arrays
};

template <typename C>
__device__ __forceinline__ C czero() {
  C z;
  z.x = 0;
  z.y = 0;
  return z;
}

// Workgroup barrier ordering LDS only.  __syncthreads() also waits for every
// outstanding global load (vmcnt(0)), which would drain the next plane's
// prefetch at each barrier; here only LDS traffic (lgkmcnt) is waited for.
// The empty asm statements keep the compiler from moving memory accesses
// across the barrier; loads still in flight are waited for where their
// registers are first used.
__device__ __forceinline__ void sync_lds() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // gfx9 encoding: vmcnt 63, expcnt 7, lgkmcnt 0
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Raw buffer loads: an offset at or beyond the buffer's size returns zero,
// which is how halo cells outside the box read as zero without a select on
// the loaded value (a select would force the wait right after the load).
// Buffers are limited to below 4 GiB (checked on the host).
constexpr unsigned kOob = 0xFFFFFFF0u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ void bload(__amdgpu_buffer_rsrc_t r, unsigned off, double2& v) {
  v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
__device__ __forceinline__ void bload(__amdgpu_buffer_rsrc_t r, unsigned off, float2& v) {
  v = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void bload(__amdgpu_buffer_rsrc_t r, unsigned off, double& v) {
  v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void bload(__amdgpu_buffer_rsrc_t r, unsigned off, float& v) {
  v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// Neighbouring lanes' values by DPP (no LDS traffic): lane i receives lane
// i - 1 (shr) or i + 1 (shl); lanes past the wave's ends receive zero.
__device__ __forceinline__ double dpp_shift(double v, bool right) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = (int)b, hi = (int)(b >> 32);
  const int l2 = right ? __builtin_amdgcn_update_dpp(0, lo, 0x138, 0xF, 0xF, true)
                       : __builtin_amdgcn_update_dpp(0, lo, 0x130, 0xF, 0xF, true);
  const int h2 = right ? __builtin_amdgcn_update_dpp(0, hi, 0x138, 0xF, 0xF, true)
                       : __builtin_amdgcn_update_dpp(0, hi, 0x130, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((long long)h2 << 32) | (unsigned)l2);
}
__device__ __forceinline__ float dpp_shift(float v, bool right) {
  const int b = __builtin_bit_cast(int, v);
  return __builtin_bit_cast(float, right ? __builtin_amdgcn_update_dpp(0, b, 0x138, 0xF, 0xF, true)
                                         : __builtin_amdgcn_update_dpp(0, b, 0x130, 0xF, 0xF, true));
}
template <typename C>
__device__ __forceinline__ C dpp_shift_c(C v, bool right) {
  C o;
  o.x = dpp_shift(v.x, right);
  o.y = dpp_shift(v.y, right);
  return o;
}
// The same, with the lane past the wave's end (lane 0 for shr, 63 for shl)
// receiving `edge` instead of zero (its destination is left as it was).
__device__ __forceinline__ double dpp_shift_edge(double v, bool right, double edge) {
  const long long b = __builtin_bit_cast(long long, v), e = __builtin_bit_cast(long long, edge);
  const int lo = (int)b, hi = (int)(b >> 32), elo = (int)e, ehi = (int)(e >> 32);
  const int l2 = right ? __builtin_amdgcn_update_dpp(elo, lo, 0x138, 0xF, 0xF, false)
                       : __builtin_amdgcn_update_dpp(elo, lo, 0x130, 0xF, 0xF, false);
  const int h2 = right ? __builtin_amdgcn_update_dpp(ehi, hi, 0x138, 0xF, 0xF, false)
                       : __builtin_amdgcn_update_dpp(ehi, hi, 0x130, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)h2 << 32) | (unsigned)l2);
}
__device__ __forceinline__ float dpp_shift_edge(float v, bool right, float edge) {
  const int b = __builtin_bit_cast(int, v), e = __builtin_bit_cast(int, edge);
  return __builtin_bit_cast(float, right ? __builtin_amdgcn_update_dpp(e, b, 0x138, 0xF, 0xF, false)
                                         : __builtin_amdgcn_update_dpp(e, b, 0x130, 0xF, 0xF, false));
}
template <typename C, typename T>
__device__ __forceinline__ C dpp_shift_edge_c(C v, bool right, T ex, T ey) {
  C o;
  o.x = dpp_shift_edge(v.x, right, ex);
  o.y = dpp_shift_edge(v.y, right, ey);
  return o;
}

// Half of the Horner step per launch:
//   half A:  u3 = psi + (dt/4) L psi,  u2 = psi + (dt/3) L u3   -> u2
//   half B:  u1 = psi + (dt/2) L u2,   psi' = psi + dt L u1      -> psi'
// w is the field the first stage differentiates (psi in A, u2 in B), base the
// Horner base psi (the same buffer in A).  Tiles are TY = 8 rows by TZ
// planes (TZ in {4, 8, 16}, chosen by the tuner) by one x chunk: the whole
// row when nx <= 128, else chunks of at most 124 output columns loaded with
// a two-column halo on each side (the chunk edges see zero neighbours, which
// only corrupts the halo columns, never an output).  12 waves.
constexpr int kTY2 = 8, kHalo2 = 2, kChunk = kCols - 2 * kHalo2;

// one box of a (possibly batched) two-stage launch
struct Box2 {
  FusedArgs a;
  const void* w;
  const void* base;
  void* out;
  const void* V;
  const double2* av;
  const double2* fb;
  double2* aux_out;
  int tile_begin;  // first global tile of this box in the launch
  int pad;
};

// KEEPD (the adjoint's Horner steps): keep1 receives the stage-1 increment
// (output minus base) instead of the output, and keep2 the stage-2 increment,
// so that differences of the intermediates carry no cancellation.
template <typename T, int ORDER, bool SAME_BASE, int TZ, int PF, bool KEEPD = false>
__device__ __forceinline__ void fused2_body(const typename cpx<T>::t* __restrict__ w_in,
                                            const typename cpx<T>::t* __restrict__ base_in,
                                            typename cpx<T>::t* __restrict__ out, const T* __restrict__ V,
                                            const FusedArgs& a, double cA, double cB,
                                            const double2* __restrict__ av, const double2* __restrict__ fb,
                                            double2* __restrict__ aux_out, int tile,
                                            typename cpx<T>::t* __restrict__ keep1 = nullptr,
                                            typename cpx<T>::t* __restrict__ keep2 = nullptr) {
  using C = typename cpx<T>::t;
  constexpr int TY = kTY2, H = kHalo2;
  constexpr int ROWS = TY + 2 * H;
  constexpr int NT = 64 * ROWS;
  constexpr int ITERS = TZ + 2 * H;
  constexpr bool FO = ORDER == 3;
  constexpr int FP = TZ + 2, FR = ROWS - 2;
  // first-order face data in LDS (sizes in double2; 1 = unused)
  constexpr int NXG = FO ? 2 * FP * FR : 1, NXF = FO ? 2 * TZ * TY : 1;
  constexpr int NYG = FO ? FP * kCols : 1, NYF = FO && !SAME_BASE ? TZ * kCols : 1;
  constexpr int NZF = FO && !SAME_BASE ? TY * kCols : 1;
  constexpr int NVX = FO ? 2 * TY * 2 : 1, NVY = FO ? 2 * kCols : 1;
  // Rows published for the y/x neighbours: the stage-1 inputs w of every row
  // and the stage-1 outputs s1 of rows 1 .. ROWS-2 (the only rows stage 2
  // reads).  Double-buffered (one barrier per plane) when both buffers fit in
  // the 160 KiB of LDS beside the face data.
  constexpr int kPlaneBytes = (2 * ROWS - 2) * 2 * 66 * (int)sizeof(C);
  constexpr int kFaceBytes = 16 * (NXG + NXF + NYG + NYF + NZF + NVX + NVY);
  constexpr int DBN = 2 * kPlaneBytes + kFaceBytes <= 160 * 1024 ? 2 : 1;
  __shared__ C plw[DBN][ROWS][2][66];
  __shared__ C pls[DBN][ROWS - 2][2][66];

  const int lane = threadIdx.x & 63;
  const int r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform row
  const int tx = tile % a.ntx, rest = tile / a.ntx;
  const int ty = rest % a.nty, tz = rest / a.nty;
  const int y0 = ty * TY, z0 = tz * TZ;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int sz = nx * ny;
  const int y = y0 - H + r;
  const bool row_in = y >= 0 && y < ny;
  const int ybase = y * nx;
  const bool own_row = r >= H && r < H + TY && row_in;
  // columns: x = xb + 2 lane + c; owned outputs in [xo, xe)
  const int xo = tx * a.xw, xe = min(xo + a.xw, nx);
  const int xb = a.ntx == 1 ? 0 : xo - H;

  for (int i = threadIdx.x; i < DBN * ROWS * 2 * 66; i += NT) (&plw[0][0][0][0])[i] = czero<C>();
  for (int i = threadIdx.x; i < DBN * (ROWS - 2) * 2 * 66; i += NT) (&pls[0][0][0][0])[i] = czero<C>();

  C Yc[2][2], Yb[2][2];  // stage inputs: centre / below (j = 0: w, j = 1: stage-1 output)
  C Bd[2][2];            // base at planes zi-1, zi-2 (separate base only)
  T Vd[2][2];            // V at planes zi-1, zi-2
  C pf[PF][2], pb[PF][2];  // fields of the next PF planes (ring indexed by plane)
  T pv[PF][2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      Yc[j][c] = Yb[j][c] = Bd[j][c] = czero<C>();
      Vd[j][c] = T(0);
    }
#pragma unroll
    for (int q = 0; q < PF; ++q) pb[q][c] = czero<C>();
  }
  const T diag = T(a.diag), off = T(a.off);
  const unsigned cbytes = (unsigned)(nz * sz) * (unsigned)sizeof(C);
  const __amdgpu_buffer_rsrc_t rw = make_rsrc(w_in, cbytes), rbase = make_rsrc(base_in, cbytes);
  const __amdgpu_buffer_rsrc_t rv = make_rsrc(V, a.has_V ? (unsigned)(nz * sz) * (unsigned)sizeof(T) : 0u);

  // plane zz into ring slot q; cells outside the box read as zero
  auto fetch = [&](int zz, int q) {
    const bool ok = row_in && zz >= 0 && zz < nz;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int x = xb + 2 * lane + c;
      const bool in = ok && x >= 0 && x < nx;
      const unsigned idx = in ? (unsigned)(zz * sz + ybase + x) : 0u;
      bload(rw, in ? idx * (unsigned)sizeof(C) : kOob, pf[q][c]);
      if (!SAME_BASE) bload(rbase, in ? idx * (unsigned)sizeof(C) : kOob, pb[q][c]);
      bload(rv, in ? idx * (unsigned)sizeof(T) : kOob, pv[q][c]);
    }
  };
#pragma unroll
  for (int q = 0; q < PF; ++q) fetch(z0 - H + q, q);

  // First order: the tile's face data, read once before the sweep.
  //  * x faces (both sides), in LDS: the auxiliary input g = av over the
  //    stage-1 planes z0-1 .. z0+TZ and rows 1 .. ROWS-2, and the base
  //    f0 = fb over the own planes and rows (the halo waves form v and the
  //    outputs).
  //  * the tile's z-face plane, if it has one (at most one when
  //    nz >= TZ + 2): each row wave holds g of its own row there in
  //    registers; f0 over the own rows is staged in LDS when the base is a
  //    separate buffer (half B) and is g itself otherwise.
  //  * the tile's y-face row, if it has one (at most one when
  //    ny >= TY + 2), in LDS: g over the stage-1 planes and, with a separate
  //    base, f0 over the own planes.  The halo waves form its stage-2 source
  //    and auxiliary outputs during the sweep, as for the x faces.
  // The stage-2 source is v = f0 + cA (b g + a w) and the auxiliary output
  // f0 + cB (b v + a s1).  Every thread issues all of its loads before using
  // any, so the staging costs one memory round trip, overlapped with the
  // first plane fetch.
  __shared__ double2 fxg[NXG];  // [side][plane][row]
  __shared__ double2 fxf[NXF];  // [side][own plane][own row]
  __shared__ double2 fyg[NYG];  // [plane][local column]
  __shared__ double2 fyf[NYF];  // [own plane][local column]
  __shared__ double2 fzf[NZF];  // [own row][local column]
  // z face: g of this wave's row at the face plane, per column
  double2 gz[2] = {make_double2(0, 0), make_double2(0, 0)};
  // auxiliary stages v of the next two planes: x faces [plane & 1][own row]
  // [side], y-face row [plane & 1][local column]
  __shared__ double2 vx[NVX];
  __shared__ double2 vy[NVY];
  int yface = -1, zface = -1;  // face index (2/3, 4/5) of the tile's y row / z plane
  // face slab offsets as scalars (a per-lane index into the argument array
  // would make the compiler loop over the distinct indices)
  const int off_x0 = a.face_off[0], off_x1 = a.face_off[1];
  int off_y = 0, off_z = 0;
  if (FO) {
    const int ylo = y0 - H + 1, zlo = z0 - 1;
    if (ylo <= 0) yface = 2;
    else if (ylo <= ny - 1 && ny - 1 < ylo + FR) yface = 3;
    if (zlo <= 0) zface = 4;
    else if (zlo <= nz - 1 && nz - 1 < zlo + FP) zface = 5;
    off_y = yface == 3 ? a.face_off[3] : a.face_off[2];
    off_z = zface == 5 ? a.face_off[5] : a.face_off[4];
    constexpr int NXA = NXG + NXF;
    constexpr int KX = (NXA + NT - 1) / NT, KYG = (NYG + NT - 1) / NT, KYF = (NYF + NT - 1) / NT;
    constexpr int KZF = (NZF + NT - 1) / NT;
    double2 rx[KX], ryg[KYG], ryf[KYF], rzf[KZF];
    if (zface >= 0 && row_in && r >= 1 && r < ROWS - 1) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int xx = xb + 2 * lane + c;
        if (xx >= 0 && xx < nx) gz[c] = av[off_z + ybase + xx];
      }
    }
#pragma unroll
    for (int j = 0; j < KX; ++j) {
      const int i = threadIdx.x + j * NT;
      rx[j] = make_double2(0, 0);
      if (i < NXG) {
        const int rr = i % FR, pl = (i / FR) % FP, side = i / (FR * FP);
        const int yy = ylo + rr, zz = zlo + pl;
        if (yy >= 0 && yy < ny && zz >= 0 && zz < nz) rx[j] = av[(side ? off_x1 : off_x0) + zz * ny + yy];
      } else if (i < NXA) {
        const int e = i - NXG;
        const int jj = e % TY, pl = (e / TY) % TZ, side = e / (TY * TZ);
        const int yy = y0 + jj, zz = z0 + pl;
        if (yy < ny && zz < nz) rx[j] = fb[(side ? off_x1 : off_x0) + zz * ny + yy];
      }
    }
#pragma unroll
    for (int j = 0; j < KYG; ++j) {
      const int i = threadIdx.x + j * NT;
      const int lx = i % kCols, pl = i / kCols;
      const int xx = xb + lx, zz = zlo + pl;
      ryg[j] = make_double2(0, 0);
      if (yface >= 0 && i < NYG && xx >= 0 && xx < nx && zz >= 0 && zz < nz) ryg[j] = av[off_y + zz * nx + xx];
    }
#pragma unroll
    for (int j = 0; j < KYF; ++j) {
      const int i = threadIdx.x + j * NT;
      const int lx = i % kCols, pl = i / kCols;
      const int xx = xb + lx, zz = z0 + pl;
      ryf[j] = make_double2(0, 0);
      if (!SAME_BASE && yface >= 0 && i < NYF && xx >= 0 && xx < nx && zz < nz) ryf[j] = fb[off_y + zz * nx + xx];
    }
#pragma unroll
    for (int j = 0; j < KZF; ++j) {
      const int i = threadIdx.x + j * NT;
      const int lx = i % kCols, jj = i / kCols;
      const int xx = xb + lx, yy = y0 + jj;
      rzf[j] = make_double2(0, 0);
      if (!SAME_BASE && zface >= 0 && i < NZF && xx >= 0 && xx < nx && yy < ny) rzf[j] = fb[off_z + yy * nx + xx];
    }
#pragma unroll
    for (int j = 0; j < KX; ++j) {
      const int i = threadIdx.x + j * NT;
      if (i < NXG) fxg[i] = rx[j];
      else if (i < NXA) fxf[i - NXG] = rx[j];
    }
#pragma unroll
    for (int j = 0; j < KYG; ++j) {
      const int i = threadIdx.x + j * NT;
      if (i < NYG) fyg[i] = ryg[j];
    }
    if constexpr (!SAME_BASE) {
#pragma unroll
      for (int j = 0; j < KYF; ++j) {
        const int i = threadIdx.x + j * NT;
        if (i < NYF) fyf[i] = ryf[j];
      }
#pragma unroll
      for (int j = 0; j < KZF; ++j) {
        const int i = threadIdx.x + j * NT;
        if (i < NZF) fzf[i] = rzf[j];
      }
    }
  }
  __syncthreads();

  // the y-face row when it is one of the tile's own rows (stage 2 and the
  // auxiliary outputs run there), as a tile row index; -1 otherwise
  int ryown = -1;
  if (FO && yface >= 0) {
    const int yf = yface == 3 ? ny - 1 : 0;
    if (yf >= y0 && yf < y0 + TY) ryown = yf - (y0 - H);
  }

#pragma unroll
  for (int it = 0; it < ITERS; ++it) {
    const int zi = z0 - H + it;
    // rows published by the previous iteration, and the buffers of the next
    auto& pw = plw[DBN == 2 ? (it & 1) : 0];
    auto& ps = pls[DBN == 2 ? (it & 1) : 0];
    auto& pwn = plw[DBN == 2 ? ((it + 1) & 1) : 0];
    auto& psn = pls[DBN == 2 ? ((it + 1) & 1) : 0];
    C prev[2];
    T vcur[2];
    C bcur[2], wm2[2];  // base at plane zi; w at plane zi - 2 (before the slide)
    const int q = it % PF;  // ring slot of plane zi (the loop is unrolled)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      prev[c] = pf[q][c];
      vcur[c] = pv[q][c];
      bcur[c] = SAME_BASE ? pf[q][c] : pb[q][c];
      wm2[c] = Yb[0][c];
    }
    if (it + PF < ITERS) fetch(zi + PF, q);
    // The halo waves' face work below runs after their prefetch is issued,
    // so that its latency overlaps the work.
    if (ORDER == 3 && (r == 0 || r == ROWS - 1) && lane < 2 * TY) {
      // First-order x faces, done by the two halo waves at the tile's edges
      // (idle in both stages), one lane per (own row, side).  They read the
      // rows published at the end of the previous iteration: pw holds w at
      // plane zi-1 and ps the stage-1 output s1 at plane zi-2.
      //  * top wave: v_f = fb_f + cA (b av_f + a w) at plane zi-1, for the
      //    next iteration's stage 2 (LDS ring);
      //  * bottom wave: the auxiliary output fb_f + cB (b v_f + a s1) at
      //    plane zi-2 (v_f from the ring, written an iteration earlier).
      const int j = lane >> 1, side = lane & 1;
      const int rj = H + j, yj = y0 + j;
      const int xf = side ? nx - 1 : 0, lxf = xf - xb;
      if (lxf >= 0 && lxf < kCols && yj < ny) {
        const int ci = lxf & 1, li = (lxf >> 1) + 1, rr = rj - 1;
        const int p1 = zi - 1, p2 = zi - 2;
        if (r == 0 && p1 >= z0 && p1 < z0 + TZ && p1 < nz) {
          const int pl = p1 - (z0 - 1);
          const double2 g = fxg[(side * FP + pl) * FR + rr];
          const double2 f0 = fxf[(side * TZ + (p1 - z0)) * TY + j];
          const C wv = pw[rj][ci][li];
          const double2 bg = cmul(a.b0, g), aw = cmul(a.a0, make_double2((double)wv.x, (double)wv.y));
          const double2 v = make_double2(f0.x + cA * (bg.x + aw.x), f0.y + cA * (bg.y + aw.y));
          vx[((p1 & 1) * TY + j) * 2 + side] = v;
        }
        if (r == ROWS - 1 && p2 >= z0 && p2 < z0 + TZ && p2 < nz && xf >= xo && xf < xe) {
          const double2 f0 = fxf[(side * TZ + (p2 - z0)) * TY + j];
          const double2 v = vx[((p2 & 1) * TY + j) * 2 + side];
          const C s1 = ps[rj - 1][ci][li];
          const double2 bv = cmul(a.b0, v), as1 = cmul(a.a0, make_double2((double)s1.x, (double)s1.y));
          aux_out[(side ? off_x1 : off_x0) + p2 * ny + yj] =
              make_double2(f0.x + cB * (bv.x + as1.x), f0.y + cB * (bv.y + as1.y));
        }
      }
    }
    if (ORDER == 3 && ryown >= 0 && (r == 0 || r == ROWS - 1)) {
      // The y-face row, by the same two halo waves over its whole width: the
      // top wave forms v = f0 + cA (b g + a w) at plane zi-1 into the ring;
      // the bottom wave writes the auxiliary output f0 + cB (b v + a s1) at
      // plane zi-2.
      const int p = r == 0 ? zi - 1 : zi - 2;
      if (p >= z0 && p < z0 + TZ && p < nz) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int lx = 2 * lane + c, x = xb + lx;
          if (x < 0 || x >= nx) continue;
          const double2 g = fyg[(p - z0 + 1) * kCols + lx];
          const double2 f0 = SAME_BASE ? g : fyf[(p - z0) * kCols + lx];
          if (r == 0) {
            const C wv = pw[ryown][c][lane + 1];
            const double2 bg = cmul(a.b0, g), aw = cmul(a.a0, make_double2((double)wv.x, (double)wv.y));
            vy[(p & 1) * kCols + lx] = make_double2(f0.x + cA * (bg.x + aw.x), f0.y + cA * (bg.y + aw.y));
          } else if (x >= xo && x < xe) {
            const double2 v = vy[(p & 1) * kCols + lx];
            const C s1 = ps[ryown - 1][c][lane + 1];
            const double2 bv = cmul(a.b0, v), as1 = cmul(a.a0, make_double2((double)s1.x, (double)s1.y));
            aux_out[off_y + p * nx + x] = make_double2(f0.x + cB * (bv.x + as1.x), f0.y + cB * (bv.y + as1.y));
          }
        }
      }
    }
    // First order: the x-face sources of this iteration's two stages, read
    // from LDS ahead of the stencil work so that their latency overlaps it.
    // Stage 1: av at plane zi-1; stage 2: v at plane zi-2 from the halo
    // wave's ring.  Every lane reads (the indices are clamped in range, and
    // do not bind in the active stages that use the values); only the lanes
    // holding a face column use them.  A branch here, or around the adds
    // below, splits the stage code into blocks that the compiler schedules
    // apart, which costs more than the extra reads and selects.
    double2 gx[2] = {make_double2(0, 0), make_double2(0, 0)};
    int cxf = -1;
    if (ORDER == 3) {
      const int x0 = xb + 2 * lane;
      cxf = (x0 == 0 || x0 == nx - 1) ? 0 : ((x0 + 1 == nx - 1) ? 1 : -1);
      const int side = x0 == 0 ? 0 : 1;
      const int rrc = min(max(r - 1, 0), FR - 1);
      const int plc = min(max(zi - z0, 0), FP - 1);
      const int jc = min(max(r - H, 0), TY - 1);
      gx[0] = fxg[(side * FP + plc) * FR + rrc];
      gx[1] = vx[(((zi - 2) & 1) * TY + jc) * 2 + side];
    }
#pragma unroll
    for (int k = 1; k <= 2; ++k) {
      const int zk = zi - k;
      const T cf = T(k == 1 ? cA : cB);
      const bool active = r >= k && r < ROWS - k && it >= 2 * k && row_in && zk >= 0 && zk < nz;
      C o[2];
      C dk[2];  // the stage's increment (KEEPD only)
      if constexpr (KEEPD) dk[0] = dk[1] = czero<C>();
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int lx = 2 * lane + c, x = xb + lx;
        const bool in = x >= 0 && x < nx;
        o[c] = czero<C>();
        if (!active) continue;
        const C cen = Yc[k - 1][c], bel = Yb[k - 1][c], abv = prev[c];
        // stage k reads rows r-1 .. r+1 of w (k = 1) or of s1 (k = 2)
        auto row = [&](int rr) -> C(&)[2][66] { return k == 1 ? pw[rr] : ps[rr - 1]; };
        const C ym = row(r - 1)[c][lane + 1];
        const C yp = row(r + 1)[c][lane + 1];
        const C xm = c == 0 ? row(r)[1][lane] : Yc[k - 1][0];
        const C xp = c == 0 ? Yc[k - 1][1] : row(r)[0][lane + 2];
        C b0;
        if (SAME_BASE) b0 = k == 1 ? Yc[0][c] : wm2[c];
        else b0 = Bd[k - 1][c];
        const T v = Vd[k - 1][c];
        T hr = diag * cen.x + off * (bel.x + abv.x + ym.x + yp.x + xm.x + xp.x) + v * cen.x;
        T hi = diag * cen.y + off * (bel.y + abv.y + ym.y + yp.y + xm.y + xp.y) + v * cen.y;
        if (ORDER == 2) {
          // zeroth-order local term nf m0 y, nf = number of faces at the
          // point (0 inside); computed for every lane without a branch, in
          // the stencil's precision
          const T nf = T((x == 0) + (x == nx - 1) + (y == 0) + (y == ny - 1) + (zk == 0) + (zk == nz - 1));
          const T m0x = T(a.m0.x), m0y = T(a.m0.y);
          hr += nf * (m0x * cen.x - m0y * cen.y);
          hi += nf * (m0x * cen.y + m0y * cen.x);
        }
        // columns outside the box stay zero (they are x neighbours)
        o[c].x = in ? b0.x + cf * hi : T(0);
        o[c].y = in ? b0.y - cf * hr : T(0);
        if constexpr (KEEPD) {
          dk[c].x = in ? cf * hi : T(0);
          dk[c].y = in ? -cf * hr : T(0);
        }
      }
      if (ORDER == 3 && active) {
        // First order: the psi stage also sees -i sum_f g_f at face points,
        // with g = the auxiliary input (stage 1) or the auxiliary stage
        // v_f = fb_f + cA (b av_f + a w) (stage 2), added to the plain stage
        // output as -i cf g.
        const int pl = zk - (z0 - 1);
        const double cf2 = k == 1 ? cA : cB;
        // x faces: at most one column per lane, its source read above,
        // added without a branch (zero for the other columns)
        {
          const double2 g = gx[k - 1];
          const bool c0 = cxf == 0, c1 = cxf == 1;
          if constexpr (std::is_same<T, double>::value) {
            o[0].x += cf2 * (c0 ? g.y : 0.0);
            o[0].y += -cf2 * (c0 ? g.x : 0.0);
            o[1].x += cf2 * (c1 ? g.y : 0.0);
            o[1].y += -cf2 * (c1 ? g.x : 0.0);
            if constexpr (KEEPD) {
              dk[0].x += cf2 * (c0 ? g.y : 0.0);
              dk[0].y += -cf2 * (c0 ? g.x : 0.0);
              dk[1].x += cf2 * (c1 ? g.y : 0.0);
              dk[1].y += -cf2 * (c1 ? g.x : 0.0);
            }
          } else {
            const T dx = T(cf2 * g.y), dy = T(-cf2 * g.x);
            o[0].x += c0 ? dx : T(0);
            o[0].y += c0 ? dy : T(0);
            o[1].x += c1 ? dx : T(0);
            o[1].y += c1 ? dy : T(0);
          }
        }
        // y and z faces: whole rows (wave-uniform), both columns of each lane,
        // sources precomputed at staging; stage 2 also writes the auxiliary
        // outputs Q + cB a s1 at owned points
        const bool fy = y == 0 || y == ny - 1, fz = zk == 0 || zk == nz - 1;
        if (fy || fz) {
          const bool own_pt = k == 2 && own_row && it >= 2 * H;
          const double2 ba = make_double2(cB * a.a0.x, cB * a.a0.y);
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const int lx = 2 * lane + c, x = xb + lx;
            if (x < 0 || x >= nx) continue;
            const bool own = own_pt && x >= xo && x < xe;
            double sr = 0, si = 0;
            double2 as1 = make_double2(0, 0);
            if (k == 2 && own) as1 = cmul(ba, make_double2((double)Yc[1][c].x, (double)Yc[1][c].y));
            // stage 1 adds g; stage 2 adds v = f0 + cA (b g + a w), w at this
            // plane, and at owned points writes f0 + cB b v + cB a s1
            const double2 wv = make_double2((double)wm2[c].x, (double)wm2[c].y);
            auto face = [&](const double2 g, const double2 f0, int oidx) {
              if (k == 1) {
                sr += g.x;
                si += g.y;
                return;
              }
              const double2 bg = cmul(a.b0, g), aw = cmul(a.a0, wv);
              const double2 v = make_double2(f0.x + cA * (bg.x + aw.x), f0.y + cA * (bg.y + aw.y));
              sr += v.x;
              si += v.y;
              if (own) {
                const double2 bv = cmul(a.b0, v);
                aux_out[oidx] = make_double2(f0.x + cB * bv.x + as1.x, f0.y + cB * bv.y + as1.y);
              }
            };
            const double2 zero = make_double2(0, 0);
            if (fy) {
              // stage 1: g; stage 2: v from the halo wave's ring (the
              // auxiliary outputs are written there too)
              const double2 g = k == 1 ? fyg[pl * kCols + lx] : vy[(zk & 1) * kCols + lx];
              sr += g.x;
              si += g.y;
            }
            if (fz) {
              const double2 f0 = SAME_BASE ? gz[c] : (k == 2 ? fzf[(r - H) * kCols + lx] : zero);
              face(gz[c], f0, off_z + y * nx + x);
            }
            o[c].x += T(cf2 * si);
            o[c].y += T(-cf2 * sr);
            if constexpr (KEEPD) {
              dk[c].x += T(cf2 * si);
              dk[c].y += T(-cf2 * sr);
            }
          }
        }
      }
      C* kp = k == 1 ? keep1 : (KEEPD ? keep2 : nullptr);
      if (kp && own_row && zk >= z0 && zk < z0 + TZ && zk < nz) {
        // the stage-1 output (or with KEEPD the stage's increment) at the
        // tile's own points, kept for the adjoint
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int x = xb + 2 * lane + c;
          C v = o[c];
          if constexpr (KEEPD) v = dk[c];
          if (x >= xo && x < xe) kp[zk * sz + ybase + x] = v;
        }
      }
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        Yb[k - 1][c] = Yc[k - 1][c];
        Yc[k - 1][c] = prev[c];
        prev[c] = o[c];
      }
    }
    const int z2 = zi - 2;
    const bool own_out = own_row && it >= 2 * H && z2 < nz;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int x = xb + 2 * lane + c;
      if (own_out && x >= xo && x < xe) out[z2 * sz + ybase + x] = prev[c];
      Vd[1][c] = Vd[0][c];
      Vd[0][c] = vcur[c];
      if (!SAME_BASE) {
        Bd[1][c] = Bd[0][c];
        Bd[0][c] = bcur[c];
      }
    }
    // publish this plane's stage inputs; with a single buffer every wave
    // must first be done reading the previous ones
    if (DBN == 1) sync_lds();
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      pwn[r][c][lane + 1] = Yc[0][c];
      if (r >= 1 && r < ROWS - 1) psn[r - 1][c][lane + 1] = Yc[1][c];
    }
    sync_lds();
  }
}

// one box, arguments in the kernel argument segment
template <typename T, int ORDER, bool SAME_BASE, int TZ, int PF = 1>
__global__ void __launch_bounds__(64 * (kTY2 + 2 * kHalo2)) fused2_kernel(
    const typename cpx<T>::t* __restrict__ w_in, const typename cpx<T>::t* __restrict__ base_in,
    typename cpx<T>::t* __restrict__ out, const T* __restrict__ V, FusedArgs a, double cA, double cB,
    const double2* __restrict__ av, const double2* __restrict__ fb, double2* __restrict__ aux_out,
    typename cpx<T>::t* __restrict__ keep1) {
  int tile = blockIdx.x;
  if (a.tiles_per_xcd) tile = (blockIdx.x & 7) * a.tiles_per_xcd + (blockIdx.x >> 3);
  fused2_body<T, ORDER, SAME_BASE, TZ, PF>(w_in, base_in, out, V, a, cA, cB, av, fb, aux_out, tile, keep1);
}

// the same keeping the stage increments (the adjoint's Horner steps)
template <typename T, int ORDER, bool SAME_BASE, int TZ>
__global__ void __launch_bounds__(64 * (kTY2 + 2 * kHalo2)) fused2_keepd_kernel(
    const typename cpx<T>::t* __restrict__ w_in, const typename cpx<T>::t* __restrict__ base_in,
    typename cpx<T>::t* __restrict__ out, const T* __restrict__ V, FusedArgs a, double cA, double cB,
    const double2* __restrict__ av, const double2* __restrict__ fb, double2* __restrict__ aux_out,
    typename cpx<T>::t* __restrict__ keep1, typename cpx<T>::t* __restrict__ keep2) {
  int tile = blockIdx.x;
  if (a.tiles_per_xcd) tile = (blockIdx.x & 7) * a.tiles_per_xcd + (blockIdx.x >> 3);
  fused2_body<T, ORDER, SAME_BASE, TZ, 1, true>(w_in, base_in, out, V, a, cA, cB, av, fb, aux_out, tile, keep1,
                                               keep2);
}

// many boxes in one launch: the grid is the concatenation of the boxes' tiles
// (padded to a multiple of 8 for the XCD-aware order); each workgroup finds
// its box by binary search over the boxes' first tiles
template <typename T, int ORDER, bool SAME_BASE, int TZ, int PF = 1>
__global__ void __launch_bounds__(64 * (kTY2 + 2 * kHalo2)) fused2_batch_kernel(
    const Box2* __restrict__ boxes, int nbox, int total_tiles, int half) {
  using C = typename cpx<T>::t;
  const int per_xcd = gridDim.x >> 3;
  const int t = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (t >= total_tiles) return;
  int lo = 0, hi = nbox - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (boxes[mid].tile_begin <= t) lo = mid;
    else hi = mid - 1;
  }
  const Box2& b = boxes[lo];
  // Horner coefficients of the box's own time step: (dt/4, dt/3) or (dt/2, dt)
  const double cA = half ? b.a.coef[2] : b.a.coef[4], cB = half ? b.a.coef[1] : b.a.coef[3];
  fused2_body<T, ORDER, SAME_BASE, TZ, PF>(static_cast<const C*>(b.w), static_cast<const C*>(b.base),
                                       static_cast<C*>(b.out), static_cast<const T*>(b.V), b.a, cA, cB, b.av, b.fb,
                                       b.aux_out, t - b.tile_begin);
}

// ---------------------------------------------------------------------------
// One-pass step: all four Horner stages in one z-marching sweep, so the
// state, the potential and the result cross HBM once per step (40 B per
// point at complex128).  The tile is the whole row (nx <= 128) by TY rows by
// TZ planes, with four-deep halos in y and z; stage k is computed on rows
// k .. ROWS-1-k and planes z0-(4-k) .. z0+TZ+(3-k), so each stage is exact
// where the next reads it.  Register state per lane (two columns): the
// centre and below planes of each stage's input, the Horner base at the two
// oldest planes and V at the four stage planes.  The stage inputs' centre
// planes are published in LDS, level j (the output of stage j, level 0 =
// psi) only on the rows stage j+1 reads, double-buffered (one barrier per
// plane).  complex128: TY = 4, TZ = 16, 12 waves (about 160 VGPRs);
// complex64: TY = 8, TZ = 8, 16 waves.
// ---------------------------------------------------------------------------
constexpr int kHalo4 = 4;
template <typename T> struct Tile4;
template <> struct Tile4<double> { static constexpr int TY = 4, TZ = 16; };
template <> struct Tile4<float> { static constexpr int TY = 8, TZ = 8; };

template <typename T>
__host__ __device__ constexpr int rows4() { return Tile4<T>::TY + 2 * kHalo4; }
// first LDS row of level j (level j holds the ROWS - 2j rows j .. ROWS-1-j)
template <typename T>
__host__ __device__ constexpr int level_base4(int j) { return j * rows4<T>() - j * (j - 1); }

// The step polynomial is applied as the product of its two real quadratic
// factors, P(x) = (1 + a1 x + b1 x^2)(1 + a2 x + b2 x^2), each in two stages
// (u = state, L = generator, D = dt):
//   stage 1: t = a1 u + b1 D L u      stage 2: v = u + D L t
//   stage 3: s = a2 v + b2 D L v      stage 4: u' = v + D L s
// The same polynomial as the Taylor sum, in another rounding order.  Every
// stage's base is its own input (stages 1, 3) or the input of the stage
// before it at the same plane (stages 2, 4), which the z queue already holds,
// so no separate copy of the step's initial state rides along.
// ORDER: 0 = zero outside the box, 2 = zeroth order (local face term),
// 3 = first order (Theorem 3.2, local face operators): the psi stage adds
// -i g_k sum_f A_f at face points (A_f the face's auxiliary stage input, g_k
// the stage's coefficient) and the auxiliary stage is base + g_k (b A + a
// psi_in), with the bases above.  A face point's auxiliary values pass
// through the four stages in four consecutive planes of the march:
//  * x faces and the tile's y-face row: helper waves (the halo rows, which
//    take part in no stage, and at a y face every row outside the box) run
//    the auxiliary stages one plane ahead of the row waves, from the stage
//    inputs published in LDS, and hand the next plane's sources A over
//    through LDS (double-buffered by plane parity); they keep the bases in
//    LDS slots indexed by plane & 3.  The jobs are split among the helpers
//    as described at the helper loop; the x faces' f0 is staged for the
//    whole march at the start, the y face's fetched a plane ahead;
//  * the z-face plane: one stage at a time is on it, so the row waves run
//    its auxiliary stage themselves (slots per thread; f0 read at stage 1).
// So the first-order tile needs ny > ROWS and nz > TZ + 4 (at most one face
// row and plane per tile), and one plane buffer (two barriers per plane) to
// fit the slots in LDS.
// FULL: every lane's two columns lie in the box (nx == 128); otherwise the
// stage outputs of columns x >= nx are forced to zero (they are read as the
// x neighbours of the last column).
template <typename T, int ORDER, bool FULL, bool DB>
__global__ void __launch_bounds__(64 * rows4<T>()) fused4_kernel(const typename cpx<T>::t* __restrict__ pin,
                                                                  typename cpx<T>::t* __restrict__ pout,
                                                                  const T* __restrict__ V, FusedArgs a,
                                                                  const double2* __restrict__ fin,
                                                                  double2* __restrict__ fout) {
  using C = typename cpx<T>::t;
  constexpr int TY = Tile4<T>::TY, TZ = Tile4<T>::TZ, H = kHalo4;
  constexpr int ROWS = rows4<T>();
  constexpr int NT = 64 * ROWS;
  constexpr int ITERS = TZ + 2 * H;
  constexpr int NLR = level_base4<T>(4);  // published rows over the four levels
  constexpr bool FO = ORDER == 3;
  // rows as [column parity][lane] (x neighbours come by DPP, so no guard
  // cells); two buffers (DB: one barrier per plane) or one (two barriers)
  __shared__ C pl[DB ? 2 : 1][NLR][2][64];
  // first-order face data (sizes in double2; 1 when unused)
  constexpr int NXF = FO ? 2 * ROWS * ITERS : 1, NXS = FO ? 2 * 4 * 2 * ROWS : 1, NXB = FO ? 2 * ROWS * 4 : 1;
  constexpr int NYS = FO ? 2 * 4 * 2 * 64 : 1, NYB = FO ? 4 * 2 * 64 : 1, NZC = FO ? ROWS * 2 * 64 * 2 : 1;
  __shared__ double2 xf0[NXF];  // [march plane][side][row]        x-face f0
  __shared__ double2 xsrc[NXS];  // [plane parity][stage][side][row] x-face stage inputs A
  __shared__ double2 xb[NXB];   // [plane & 3][side][row]          x-face bases
  __shared__ double2 ysrc[NYS];  // [plane parity][stage][c][lane]  y-face stage inputs A
  __shared__ double2 yb[NYB];   // [plane & 3][c][lane]            y-face bases
  __shared__ double2 zch[NZC];  // [row][c][A, base][lane]         z-face slots

  const int lane = threadIdx.x & 63;
  const int r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform row
  // an orbital batch: blockIdx.y picks the orbital's arrays (V is shared)
  pin += (long long)blockIdx.y * a.bstride;
  pout += (long long)blockIdx.y * a.bstride;
  if (FO) {
    fin += (long long)blockIdx.y * a.fstride;
    fout += (long long)blockIdx.y * a.fstride;
  }
  int tile = blockIdx.x;
  if (a.tiles_per_xcd) tile = (blockIdx.x & 7) * a.tiles_per_xcd + (blockIdx.x >> 3);
  const int ty = tile % a.nty, tz = tile / a.nty;
  const int y0 = ty * TY, z0 = tz * TZ;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int sz = nx * ny;
  const int y = y0 - H + r;
  const bool row_in = y >= 0 && y < ny;
  const int ybase = y * nx;
  const bool own_row = r >= H && r < H + TY && row_in;
  bool inx[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) inx[c] = FULL || 2 * lane + c < nx;

  for (int i = threadIdx.x; i < (DB ? 2 : 1) * NLR * 2 * 64; i += NT) (&pl[0][0][0][0])[i] = czero<C>();

  // first order: the faces the tile meets
  const int xh = nx - 1;  // high x-face column
  int yrow = -1, yface = -1;  // the tile row on a y face, and the face
  int zface_plane = -1, zface = -1;  // the z-face plane the march meets
  if (FO) {
    if (y0 - H <= 0) yrow = H - y0, yface = 2;
    else if (y0 - H + ROWS - 1 >= ny - 1) yrow = ny - 1 - (y0 - H), yface = 3;
    if (yrow < 1 || yrow > ROWS - 2) yrow = yface = -1;  // no stage runs on rows 0 and ROWS-1
    if (z0 - H <= 0) zface_plane = 0, zface = 4;
    else if (z0 + TZ + H - 1 >= nz - 1) zface_plane = nz - 1, zface = 5;
    // the x-face f0 over the march
    for (int i = threadIdx.x; i < NXF; i += NT) {
      const int q = i % ITERS, rr = (i / ITERS) % ROWS, side = i / (ITERS * ROWS);
      const int yy = y0 - H + rr, zz = z0 - H + q;
      double2 v = make_double2(0, 0);
      if (yy >= 0 && yy < ny && zz >= 0 && zz < nz) v = fin[a.face_off[side] + zz * ny + yy];
      xf0[(q * 2 + side) * ROWS + rr] = v;
    }
  }
  // Helper waves run in a loop of their own: the halo rows 0 and ROWS-1
  // (which take part in no stage) publish their psi row, and with the first
  // order every wave whose row lies outside the box (tiles at a y face) joins
  // them for the face jobs, the auxiliary stages of the plane's four stages:
  //  * without a y-face row (two helpers): helper 0 runs the x faces' stages
  //    1-2, helper 1 stages 3-4, one (stage, side, row) item per lane;
  //  * with one and at least five helpers: helpers 0-3 run the y-face row's
  //    stages 1-4 (two columns per lane), helper 4 all x-face items;
  //  * otherwise (a y-face row in a tile's halo, few helpers): helper 0 the
  //    stages 1-2 of both, the last helper stages 3-4.
  // Rows 0 and ROWS-1 also fetch the y face's f0 (even / odd columns).
  const int nlo = FO ? min(max(H - y0, 1), ROWS) : 1;            // rows 0 .. nlo-1
  const int hstart = FO ? min(max(ny - y0 + H, 0), ROWS - 1) : ROWS - 1;  // rows hstart ..
  const bool helper = r < nlo || r >= hstart;
  constexpr int NXI = FO ? 4 * 2 * ROWS : 0;           // x-face items
  const int ycol = r == 0 ? 0 : 1;                     // f0 fetch of the y face
  const bool yfetch = FO && yrow >= 0 && (r == 0 || r == ROWS - 1) && 2 * lane + ycol < nx;

  C Yc[4][2], Yb[4][2];  // stage-k inputs (level k-1): centre / below plane
  T Dd[4][2];            // diagonal of H (stencil centre + V) at planes zi-1 .. zi-4
  C pf[2];               // psi and V of the next plane, fetched an iteration ahead
  T pv[2];
  double2 pfy;           // y-face job: the face's f0 at the next plane (the wave's column)
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Yc[j][c] = Yb[j][c] = czero<C>();
      Dd[j][c] = T(0);
    }
  }
  pfy = make_double2(0, 0);
  const T diag = T(a.diag), off = T(a.off);
  const T sa1 = T(a.sa1), sa2 = T(a.sa2);
  const unsigned cbytes = (unsigned)(nz * sz) * (unsigned)sizeof(C);
  const __amdgpu_buffer_rsrc_t rp = make_rsrc(pin, cbytes);
  const __amdgpu_buffer_rsrc_t rv = make_rsrc(V, a.has_V ? (unsigned)(nz * sz) * (unsigned)sizeof(T) : 0u);
  const __amdgpu_buffer_rsrc_t rf = make_rsrc(fin, FO ? (unsigned)a.face_off[6] * 16u : 0u);
  // plane zz (and, for the y-face job, the face's f0 there); cells outside
  // the box read as zero (out-of-range offsets)
  auto fetch = [&](int zz, bool face_f0) __attribute__((always_inline)) {
    const bool ok = row_in && zz >= 0 && zz < nz;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const bool in = ok && inx[c];
      const unsigned idx = (unsigned)(zz * sz + ybase + 2 * lane + c);
      bload(rp, in ? idx * (unsigned)sizeof(C) : kOob, pf[c]);
      bload(rv, in ? idx * (unsigned)sizeof(T) : kOob, pv[c]);
    }
    if (FO && face_f0 && yfetch) {
      const bool okf = zz >= 0 && zz < nz;
      const unsigned fi = (unsigned)(a.face_off[yface] + zz * nx + 2 * lane + ycol);
      bload(rf, okf ? fi * 16u : kOob, pfy);
    }
  };
  fetch(z0 - H, true);
  __syncthreads();

  // one face point's auxiliary stage k: A its input, B the carried base,
  // ce the psi stage input there; returns the output and the next base
  auto aux_stage = [&](int k, double2 A, double2 B, double2 ce, double2& nB) __attribute__((always_inline)) {
    const double gk = a.coef[5 - k];
    const double2 bA = cmul(a.b0, A), ac = cmul(a.a0, ce);
    double2 base;
    if (k == 1 || k == 3) {
      const double sc = k == 1 ? a.sa1 : a.sa2;
      base = make_double2(sc * A.x, sc * A.y);
    } else {
      base = B;
    }
    const double2 nA = make_double2(base.x + gk * (bA.x + ac.x), base.y + gk * (bA.y + ac.y));
    nB = (k == 1 || k == 3) ? A : nA;  // f0 for stage 2, v for stage 4
    return nA;
  };

  if (helper) {
    const int nhelp = nlo + (ROWS - hstart);
    const int hid = r < nlo ? r : nlo + (r - hstart);
    // this helper's stages: x faces [xk0, xk1], the y-face row [yk0, yk1]
    int xk0 = 1, xk1 = 0, yk0 = 1, yk1 = 0;
    if (FO) {
      const bool yf = yrow >= 0;
      if (yf && nhelp >= 5) {
        if (hid < 4) yk0 = yk1 = hid + 1;
        else if (hid == 4) xk0 = 1, xk1 = 4;
      } else if (hid == 0) {
        xk0 = 1, xk1 = 2;
        if (yf) yk0 = 1, yk1 = 2;
      } else if (hid == nhelp - 1) {
        xk0 = 3, xk1 = 4;
        if (yf) yk0 = 3, yk1 = 4;
      }
    }
    const int nxi = (xk1 - xk0 + 1) * 2 * ROWS;  // x items of this helper
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
      const int zi = z0 - H + it;
      const auto& rd = pl[DB ? (it & 1) : 0];
      auto& wr = pl[DB ? ((it + 1) & 1) : 0];
      const int par = it & 1, npar = (it + 1) & 1;
      C cur[2];          // psi of this row at plane zi (published below)
      const double2 fy = pfy;  // y-face f0 at plane zi (the next plane's stage 1)
#pragma unroll
      for (int c = 0; c < 2; ++c) cur[c] = pf[c];
      if (it + 1 < ITERS) fetch(zi + 1, true);
      if (FO) {
        // one item: the auxiliary stage k of a face point; loads first for
        // every item of a group, then the arithmetic and the stores (the
        // items are independent: each stage is at its own plane and slot)
        struct Item {
          double2 A, B, ce;
        };
        // x faces: item j = (stage xk0 + j / (2 ROWS), side, row), two rounds
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int jj = lane + 64 * q;
          if (jj < nxi) {
            const int k = xk0 + jj / (2 * ROWS), ch = jj % (2 * ROWS), side = ch / ROWS, row = ch % ROWS;
            const int zk = zi - k;
            const int yy = y0 - H + row;
            const int xcol = side ? xh : 0;
            const int lb = level_base4<T>(k - 1) - (k - 1);
            const int rr = min(max(row, k - 1), ROWS - k);  // a published row of level k-1
            const int bi = ((zk & 3) * 2 + side) * ROWS + row;
            const C ce = rd[lb + rr][xcol & 1][xcol >> 1];
            const Item in{xsrc[((par * 4 + (k - 1)) * 2 + side) * ROWS + row], xb[bi],
                          make_double2((double)ce.x, (double)ce.y)};
            const bool act = row >= k && row < ROWS - k && it >= 2 * k && yy >= 0 && yy < ny && zk >= 0 && zk < nz;
            if (act) {
              double2 nB;
              const double2 nA = aux_stage(k, in.A, in.B, in.ce, nB);
              if (k < 4) {
                xsrc[((npar * 4 + k) * 2 + side) * ROWS + row] = nA;
                xb[bi] = nB;
              } else if (row >= H && row < H + TY && zk >= z0 && zk < z0 + TZ) {
                fout[a.face_off[side] + zk * ny + yy] = nA;
              }
            }
            // the stage-1 input of the next plane (zi): f0
            if (k == 1) xsrc[((npar * 4 + 0) * 2 + side) * ROWS + row] = xf0[(it * 2 + side) * ROWS + row];
          }
        }
        // the y-face row: stages [yk0, yk1], both columns of the lane
        for (int k = yk0; k <= yk1; ++k) {
          const int zk = zi - k;
          const int lb = level_base4<T>(k - 1) - (k - 1);
          const int rr = min(max(yrow, k - 1), ROWS - k);
          Item in[2];
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const C ce = rd[lb + rr][c][lane];
            in[c] = Item{ysrc[((par * 4 + (k - 1)) * 2 + c) * 64 + lane], yb[((zk & 3) * 2 + c) * 64 + lane],
                         make_double2((double)ce.x, (double)ce.y)};
          }
          const bool act = yrow >= k && yrow < ROWS - k && it >= 2 * k && zk >= 0 && zk < nz;
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            if (!act || !inx[c]) continue;
            double2 nB;
            const double2 nA = aux_stage(k, in[c].A, in[c].B, in[c].ce, nB);
            if (k < 4) {
              ysrc[((npar * 4 + k) * 2 + c) * 64 + lane] = nA;
              yb[((zk & 3) * 2 + c) * 64 + lane] = nB;
            } else if (yrow >= H && yrow < H + TY && zk >= z0 && zk < z0 + TZ) {
              fout[a.face_off[yface] + zk * nx + 2 * lane + c] = nA;
            }
          }
        }
        if (yfetch) ysrc[((npar * 4 + 0) * 2 + ycol) * 64 + lane] = fy;
      }
      if (!DB) sync_lds();
      if (r == 0 || r == ROWS - 1) {
#pragma unroll
        for (int c = 0; c < 2; ++c) wr[r == 0 ? 0 : level_base4<T>(1) - 1][c][lane] = cur[c];
      }
      sync_lds();
    }
    return;
  }

#pragma unroll
  for (int it = 0; it < ITERS; ++it) {
    const int zi = z0 - H + it;
    const auto& rd = pl[DB ? (it & 1) : 0];
    auto& wr = pl[DB ? ((it + 1) & 1) : 0];
    const int par = it & 1;
    C prev[2];   // the previous stage's output at the plane above (stage 1: psi(zi))
    T dcur[2];
    C ub[2];     // stage-2 base: psi at plane zi - 2
    C vb[2];     // stage-4 base: the stage-2 output at plane zi - 4
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      prev[c] = pf[c];
      dcur[c] = diag + pv[c];
      ub[c] = Yb[0][c];
      vb[c] = Yb[2][c];
    }
    if (it + 1 < ITERS) fetch(zi + 1, false);
#pragma unroll
    for (int k = 1; k <= 4; ++k) {
      const int zk = zi - k;
      const T cf = T(a.coef[5 - k]);
      const bool active = r >= k && r < ROWS - k && it >= 2 * k && row_in && zk >= 0 && zk < nz;
      C o[2];
      if (active) {
        // level k-1 rows r-1, r, r+1 (published at the end of the previous plane)
        const int lb = level_base4<T>(k - 1) - (k - 1);
        // First order on full rows: the x-face sources -i g A enter as the
        // x neighbours outside the box of columns 0 and 127, A / off (the
        // lanes past the wave's ends of the DPP shifts), so that no select is
        // needed.  Other rows add them below.
        T e0x = T(0), e0y = T(0), e1x = T(0), e1y = T(0);
        if (FO && FULL) {
          const double2 s0 = xsrc[((par * 4 + (k - 1)) * 2 + 0) * ROWS + r];
          const double2 s1 = xsrc[((par * 4 + (k - 1)) * 2 + 1) * ROWS + r];
          const double io = 1.0 / a.off;
          e0x = T(s0.x * io), e0y = T(s0.y * io), e1x = T(s1.x * io), e1y = T(s1.y * io);
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int x = 2 * lane + c;
          const C cen = Yc[k - 1][c], bel = Yb[k - 1][c], abv = prev[c];
          const C ym = rd[lb + r - 1][c][lane];
          const C yp = rd[lb + r + 1][c][lane];
          // x neighbours: the lane's other column, or the neighbouring lane's
          // (a row is one wave, so by DPP)
          C xm, xp;
          if (FO && FULL) {
            xm = c == 0 ? dpp_shift_edge_c(Yc[k - 1][1], true, e0x, e0y) : Yc[k - 1][0];
            xp = c == 0 ? Yc[k - 1][1] : dpp_shift_edge_c(Yc[k - 1][0], false, e1x, e1y);
          } else {
            xm = c == 0 ? dpp_shift_c(Yc[k - 1][1], true) : Yc[k - 1][0];
            xp = c == 0 ? Yc[k - 1][1] : dpp_shift_c(Yc[k - 1][0], false);
          }
          const T d = Dd[k - 1][c];
          T hr = d * cen.x + off * (((bel.x + abv.x) + (ym.x + yp.x)) + (xm.x + xp.x));
          T hi = d * cen.y + off * (((bel.y + abv.y) + (ym.y + yp.y)) + (xm.y + xp.y));
          if (ORDER == 2) {
            const T nf = T((x == 0) + (x == nx - 1) + (y == 0) + (y == ny - 1) + (zk == 0) + (zk == nz - 1));
            const T m0x = T(a.m0.x), m0y = T(a.m0.y);
            hr += nf * (m0x * cen.x - m0y * cen.y);
            hi += nf * (m0x * cen.y + m0y * cen.x);
          }
          if (k == 1 || k == 3) {
            const T sa = k == 1 ? sa1 : sa2;
            o[c].x = sa * cen.x + cf * hi;
            o[c].y = sa * cen.y - cf * hr;
          } else {
            const C b = k == 2 ? ub[c] : vb[c];
            o[c].x = b.x + cf * hi;
            o[c].y = b.y - cf * hr;
          }
        }
        if (FO) {
          // face sources -i g_k A_f, in FP64
          const double gk = a.coef[5 - k];
          // x faces on rows that do not fill the wave: every lane reads both
          // sides' inputs of its row (one address per wave) and adds them
          // under selects at the face columns
          if (!FULL) {
            const double2 s0 = xsrc[((par * 4 + (k - 1)) * 2 + 0) * ROWS + r];
            const double2 s1 = xsrc[((par * 4 + (k - 1)) * 2 + 1) * ROWS + r];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              const int x = 2 * lane + c;
              const double sr = (x == 0 ? s0.x : 0.0) + (x == xh ? s1.x : 0.0);
              const double si = (x == 0 ? s0.y : 0.0) + (x == xh ? s1.y : 0.0);
              o[c].x += T(gk * si);
              o[c].y -= T(gk * sr);
            }
          }
          // the tile's y-face row (whole wave)
          if (r == yrow) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              const double2 A = ysrc[((par * 4 + (k - 1)) * 2 + c) * 64 + lane];
              o[c].x += T(gk * A.y);
              o[c].y -= T(gk * A.x);
            }
          }
          // the z-face plane (wave-uniform: one stage at a time is on it)
          if (zk == zface_plane) {
            const bool own_pt = k == 4 && own_row && zk >= z0 && zk < z0 + TZ;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              if (!inx[c]) continue;
              const C ce = Yc[k - 1][c];
              const int si = (r * 2 + c) * 128 + lane;  // A at si, base at si + 64
              const double2 A = k == 1 ? fin[a.face_off[zface] + ybase + 2 * lane + c] : zch[si];
              const double2 B = k == 1 ? A : zch[si + 64];
              o[c].x += T(gk * A.y);
              o[c].y -= T(gk * A.x);
              double2 nB;
              const double2 nA = aux_stage(k, A, B, make_double2((double)ce.x, (double)ce.y), nB);
              if (k < 4) {
                zch[si] = nA;
                zch[si + 64] = nB;
              } else if (own_pt) {
                fout[a.face_off[zface] + ybase + 2 * lane + c] = nA;
              }
            }
          }
        }
#pragma unroll
        for (int c = 0; c < 2; ++c)
          if (!FULL && !inx[c]) o[c] = czero<C>();
      } else {
        o[0] = o[1] = czero<C>();
      }
      // stage k is the last reader of its input window: slide it
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        Yb[k - 1][c] = Yc[k - 1][c];
        Yc[k - 1][c] = prev[c];
        prev[c] = o[c];
      }
      // keep the next stage's LDS reads below this stage's arithmetic (with
      // all four stages' reads hoisted the registers run out)
      __builtin_amdgcn_sched_barrier(0);
    }
    // stage 4's output is the new state at plane zi - 4
    const int z4 = zi - 4;
    const bool own_out = own_row && it >= 2 * H && z4 < nz;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (own_out && inx[c]) pout[z4 * sz + ybase + 2 * lane + c] = prev[c];
      Dd[3][c] = Dd[2][c];
      Dd[2][c] = Dd[1][c];
      Dd[1][c] = Dd[0][c];
      Dd[0][c] = dcur[c];
    }
    // publish the next plane's stage inputs: level j on rows j .. ROWS-1-j
    // (with one buffer, after every wave is done reading it)
    if (!DB) sync_lds();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (r >= j && r < ROWS - j) {
        const int lr = level_base4<T>(j) + r - j;
#pragma unroll
        for (int c = 0; c < 2; ++c) wr[lr][c][lane] = Yc[j][c];
      }
    }
    sync_lds();
  }
}

template <typename T>
FusedArgs make_args4(const abc_launch& L) {
  FusedArgs a{};
  a.nx = L.g.nx;
  a.ny = L.g.ny;
  a.nz = L.g.nz;
  a.ntx = 1;
  a.xw = a.nx;
  a.nty = (a.ny + Tile4<T>::TY - 1) / Tile4<T>::TY;
  const int ntz = (a.nz + Tile4<T>::TZ - 1) / Tile4<T>::TZ;
  a.ntiles = a.nty * ntz;
  a.tiles_per_xcd = (a.ntiles % 8 == 0) ? a.ntiles / 8 : 0;
  const double s = 1.0 / (2.0 * L.h * L.h);
  a.diag = -3.0 * L.c[0] * s;
  a.off = -L.c[1] * s;
  // stage k reads coef[5 - k]: the factored form's coefficients
  a.coef[4] = L.fused_b1 * L.dt;
  a.coef[3] = L.dt;
  a.coef[2] = L.fused_b2 * L.dt;
  a.coef[1] = L.dt;
  a.coef[0] = 0;
  a.sa1 = L.fused_a1;
  a.sa2 = L.fused_a2;
  for (int f = 0; f < 7; ++f) a.face_off[f] = (int)L.g.face_off[f];
  a.m0 = L.fused_m0;
  a.b0 = L.fused_b0;
  a.a0 = L.a_loc[0];
  return a;
}

template <typename T>
FusedArgs make_args(const abc_launch& L) {
  FusedArgs a{};
  a.nx = L.g.nx;
  a.ny = L.g.ny;
  a.nz = L.g.nz;
  const int TY = kTY2, TZ = L.fused_tz;
  a.ntx = a.nx > kCols ? (a.nx + kChunk - 1) / kChunk : 1;
  a.xw = (a.nx + a.ntx - 1) / a.ntx;
  a.nty = (a.ny + TY - 1) / TY;
  const int ntz = (a.nz + TZ - 1) / TZ;
  a.ntiles = a.ntx * a.nty * ntz;
  a.tiles_per_xcd = (a.ntiles % 8 == 0) ? a.ntiles / 8 : 0;
  const double s = 1.0 / (2.0 * L.h * L.h);
  a.diag = -3.0 * L.c[0] * s;
  a.off = -L.c[1] * s;
  for (int k = 1; k <= 4; ++k) a.coef[k] = L.dt / k;
  for (int f = 0; f < 7; ++f) a.face_off[f] = (int)L.g.face_off[f];
  a.m0 = L.fused_m0;
  a.b0 = L.fused_b0;
  a.a0 = L.a_loc[0];
  return a;
}

// launch one two-stage kernel instance for a runtime tile depth
template <typename T, int ORDER, bool SB, typename... A>
void launch2(abc_timer* tm, const char* label, int tz, dim3 g, dim3 b, hipStream_t st, A... args) {

  if constexpr (ORDER == 3) {
    if (tz == 4) return abc_launch_kernel(tm, label, fused2_kernel<T, ORDER, SB, 4>, g, b, st, args...);
    return abc_launch_kernel(tm, label, fused2_kernel<T, ORDER, SB, 8>, g, b, st, args...);
  } else {
    if (tz == 4) return abc_launch_kernel(tm, label, fused2_kernel<T, ORDER, SB, 4>, g, b, st, args...);
    if (tz == 16) return abc_launch_kernel(tm, label, fused2_kernel<T, ORDER, SB, 16>, g, b, st, args...);
    return abc_launch_kernel(tm, label, fused2_kernel<T, ORDER, SB, 8>, g, b, st, args...);
  }
}

template <typename T, int ORDER, bool SB, typename... A>
void launch2_keepd(int tz, dim3 g, dim3 b, hipStream_t st, A... args) {
  if constexpr (ORDER == 3) {
    if (tz == 4) return abc_launch_kernel(nullptr, "", fused2_keepd_kernel<T, ORDER, SB, 4>, g, b, st, args...);
    return abc_launch_kernel(nullptr, "", fused2_keepd_kernel<T, ORDER, SB, 8>, g, b, st, args...);
  } else {
    if (tz == 4) return abc_launch_kernel(nullptr, "", fused2_keepd_kernel<T, ORDER, SB, 4>, g, b, st, args...);
    if (tz == 16) return abc_launch_kernel(nullptr, "", fused2_keepd_kernel<T, ORDER, SB, 16>, g, b, st, args...);
    return abc_launch_kernel(nullptr, "", fused2_keepd_kernel<T, ORDER, SB, 8>, g, b, st, args...);
  }
}

template <typename T, int ORDER, bool SB>
void launch2_batch(abc_timer* tm, const char* label, int tz, dim3 g, hipStream_t st, const Box2* boxes, int nbox,
                   int total, int half) {
  const dim3 b(64 * (kTY2 + 2 * kHalo2));
  if constexpr (ORDER == 3) {
    if (tz == 4) return abc_launch_kernel(tm, label, fused2_batch_kernel<T, ORDER, SB, 4>, g, b, st, boxes, nbox, total, half);
    return abc_launch_kernel(tm, label, fused2_batch_kernel<T, ORDER, SB, 8>, g, b, st, boxes, nbox, total, half);
  } else {
    if (tz == 4) return abc_launch_kernel(tm, label, fused2_batch_kernel<T, ORDER, SB, 4>, g, b, st, boxes, nbox, total, half);
    if (tz == 16) return abc_launch_kernel(tm, label, fused2_batch_kernel<T, ORDER, SB, 16>, g, b, st, boxes, nbox, total, half);
    return abc_launch_kernel(tm, label, fused2_batch_kernel<T, ORDER, SB, 8>, g, b, st, boxes, nbox, total, half);
  }
}

}  // namespace

int fused_max_tz(int order, int nz) {
  // first order: one z-face plane per tile needs nz >= TZ + 2
  if (order == ABC_FIRST) return nz >= 10 ? 8 : 4;
  return 16;
}

bool fused_supported(const abc_params& p, std::string* why) {
  auto no = [&](const char* m) {
    if (why) *why = m;
    return false;
  };
  if (p.radius != 1) return no("radius 1 only");
  if (p.batch > 64) return no("at most 64 orbitals");
  if (p.order == ABC_PERIODIC) return no("periodic boxes use the staged path");
  if (p.order == ABC_SECOND) return no("the second order (box form) uses the staged path");
  if ((p.order == ABC_ZEROTH || p.order == ABC_FIRST) && (p.form != ABC_FORM_FACES || p.window != 0))
    return no("local (window 0) face operators only");
  if (p.nz < 5 || p.ny < 4 || p.nx < 4) return no("nx, ny >= 4 and nz >= 5");
  if (p.order == ABC_FIRST && (p.ny < kTY2 + 2 || p.nz < 6))
    return no("first order: ny >= 10 and nz >= 6 (one y-face row and one z-face plane per tile)");
  if ((long long)p.nx * p.ny * p.nz >= (1LL << 31)) return no("grid below 2^31 points");
  // raw buffer loads address each array with 32-bit byte offsets
  if ((long long)p.nx * p.ny * p.nz * (p.dtype == ABC_C64 ? 8 : 16) >= (1LL << 32) - 16)
    return no("state array below 4 GiB");
  return true;
}

bool fused_shell_case(const abc_params& p) {
  return p.order == ABC_FIRST && p.form == ABC_FORM_FACES && p.window > 0;
}

bool fused4_supported(const abc_params& p, std::string* why) {
  auto no = [&](const char* m) {
    if (why) *why = m;
    return false;
  };
  if (fused_shell_case(p)) {
    // the condition-free sweep plus the boundary-shell rounds: the sweep's
    // own limits, R = 1 and one orbital
    if (p.radius != 1) return no("one-pass sweep with a windowed face operator: radius 1 only");
    if (p.batch != 1 || p.meanfield != ABC_MF_NONE) return no("one-pass sweep: one orbital, no mean field");
    abc_params q = p;
    q.order = ABC_DIRICHLET;
    q.window = 0;
    return fused4_supported(q, why);
  }
  if (!fused_supported(p, why)) return false;
  if (p.nx > kCols) return no("one-pass sweep: nx <= 128");
  if (p.order == ABC_FIRST) {
    // at most one y-face row and one z-face plane per tile
    const bool c64 = p.dtype == ABC_C64;
    const int rows = c64 ? rows4<float>() : rows4<double>();
    const int tz = c64 ? Tile4<float>::TZ : Tile4<double>::TZ;
    if (p.ny <= rows || p.nz <= tz + kHalo4)
      return no("one-pass sweep, first order: ny > rows per tile and nz > planes per tile + 4");
  }
  return true;
}

// The Taylor-4 polynomial 1 + x + x^2/2 + x^3/6 + x^4/24 as the product of
// two real quadratics (1 + a1 x + b1 x^2)(1 + a2 x + b2 x^2): 24 P(x) =
// (x^2 + p x + q)(x^2 + (4 - p) x + 24/q) pairs its two conjugate root
// pairs, with (p, q) solving q + 24/q + p (4 - p) = 12 and
// 24 p / q + (4 - p) q = 24 (matching the x^2 and x coefficients; x^3 and
// x^0 hold by construction).  Newton's method from (3.5, 3.8); a_i = p_i/q_i,
// b_i = 1/q_i.  Returns false unless the product reproduces every
// coefficient to 1e-14.
bool taylor4_quadratic_factors(double* a1, double* b1, double* a2, double* b2) {
  double p = 3.5, q = 3.8;
  for (int it = 0; it < 50; ++it) {
    const double f1 = q + 24.0 / q + p * (4.0 - p) - 12.0;
    const double f2 = 24.0 * p / q + (4.0 - p) * q - 24.0;
    const double j11 = 4.0 - 2.0 * p, j12 = 1.0 - 24.0 / (q * q);
    const double j21 = 24.0 / q - q, j22 = -24.0 * p / (q * q) + (4.0 - p);
    const double det = j11 * j22 - j12 * j21;
    if (det == 0) return false;
    const double dp = (f1 * j22 - f2 * j12) / det, dq = (j11 * f2 - j21 * f1) / det;
    p -= dp;
    q -= dq;
    if (std::fabs(dp) + std::fabs(dq) < 1e-16 * (std::fabs(p) + std::fabs(q))) break;
  }
  const double p2 = 4.0 - p, q2 = 24.0 / q;
  *a1 = p / q;
  *b1 = 1.0 / q;
  *a2 = p2 / q2;
  *b2 = 1.0 / q2;
  // (1 + a1 x + b1 x^2)(1 + a2 x + b2 x^2) against 1, 1, 1/2, 1/6, 1/24
  const double c1 = *a1 + *a2, c2 = *b1 + *b2 + *a1 * *a2, c3 = *a1 * *b2 + *a2 * *b1, c4 = *b1 * *b2;
  return std::fabs(c1 - 1.0) < 1e-14 && std::fabs(c2 - 0.5) < 1e-14 && std::fabs(c3 - 1.0 / 6) < 1e-14 &&
         std::fabs(c4 - 1.0 / 24) < 1e-14;
}

abc_status fused_prepare(const abc_params& p, abc_launch& L, std::vector<void*>* allocs, size_t* bytes,
                         std::string& err) {
  // the one-pass sweep where it covers the parameters (automatic path) or
  // when asked for, else two launches of two Horner stages per step, whose
  // tile depth (4, 8 or 16 planes) starts at 8 and is set by the tuner
  L.fused_stages = 2;
  // Automatic choice: the one-pass sweep wherever it covers the parameters,
  // except the first order on rows narrower than 128 columns, where its
  // x-face sources need selects and it measured slower than the two-stage
  // kernels (96^3: 48 against 39 us per step)
  // (a windowed first-order operator takes the one-pass sweep with the
  // boundary-shell rounds only when asked for: at 128^3 it measured level
  // with the staged path, w = 8 145 against 141 us per step, exact sections
  // 182 against 185)
  // Orbital batches and the mean field (orbitals as boxes of one launch):
  // the one-pass sweep for complex64 (the 96^3 x 32-orbital TDHF batch: 0.61
  // against 0.70 ms per step); complex128 measured level (0.95 against 0.94)
  // and stays on the two-stage kernels.
  const bool orbitals = p.batch > 1 || p.meanfield != ABC_MF_NONE;
  const bool auto4 = fused4_supported(p, nullptr) && !fused_shell_case(p) &&
                     (orbitals ? p.dtype == ABC_C64 : (p.order != ABC_FIRST || p.nx == kCols));
  L.fused_shell = 0;
  if (p.path == ABC_PATH_ONEPASS || (p.path == ABC_PATH_AUTO && auto4)) {
    if (!fused4_supported(p, &err)) return ABC_ENOTSUP;
    if (!taylor4_quadratic_factors(&L.fused_a1, &L.fused_b1, &L.fused_a2, &L.fused_b2)) {
      err = "one-pass sweep: factoring the Taylor polynomial failed";
      return ABC_EDEVICE;
    }
    L.fused_stages = 4;
    if (fused_shell_case(p)) {
      // four psi-sized and two face-aux buffers for the boundary-shell rounds
      L.fused_shell = 1;
      const size_t vb = (size_t)L.g.npts * (p.dtype == ABC_C64 ? 8 : 16);
      const size_t fb = (size_t)L.g.face_off[6] * sizeof(double2);
      for (int i = 0; i < 6; ++i) {
        void* ptr = nullptr;
        const size_t nb = i < 4 ? vb : fb;
        if (hipMalloc(&ptr, nb) != hipSuccess) {
          err = "one-pass sweep: boundary-shell buffers";
          return ABC_ENOMEM;
        }
        allocs->push_back(ptr);
        *bytes += nb;
        if (i < 4) L.shell.vol[i] = ptr;
        else L.shell.face[i - 4] = static_cast<double2*>(ptr);
      }
    }
  }
  L.fused_tz = std::min(8, fused_max_tz(p.order, p.nz));
  return ABC_OK;
}

bool fused_tz_valid(const abc_launch& L, int tz) {
  return (tz == 4 || tz == 8 || tz == 16) && tz <= fused_max_tz(L.order, L.g.nz);
}

namespace {

// One launch per step on the one-pass sweep; the ping-pong is arranged so
// that the last step writes the caller's buffers.
template <typename T, int ORDER>
void launch4(abc_timer* tm, bool full, dim3 g, dim3 b, hipStream_t st, const typename cpx<T>::t* src,
             typename cpx<T>::t* dst, const T* V, const FusedArgs& a, const double2* fin, double2* fout) {
  // first order: one plane buffer, so the face slots fit in LDS
  constexpr bool DB = ORDER != 3;
  if (full) abc_launch_kernel(tm, "fused_step", fused4_kernel<T, ORDER, true, DB>, g, b, st, src, dst, V, a, fin, fout);
  else abc_launch_kernel(tm, "fused_step", fused4_kernel<T, ORDER, false, DB>, g, b, st, src, dst, V, a, fin, fout);
}

template <typename T>
hipError_t step4_t(const abc_launch& L, const abc_scratch& S, void* psi_v, double2* aux, const void* V_v, int n,
                   hipStream_t st, abc_timer* tm) {
  using C = typename cpx<T>::t;
  FusedArgs a = make_args4<T>(L);
  a.has_V = V_v != nullptr;
  C* user = static_cast<C*>(psi_v);
  C* scr = static_cast<C*>(S.y[0]);
  C* src = user;
  C* dst = scr;
  const bool first = L.order == ABC_FIRST;
  double2* fsrc = aux;
  double2* fdst = S.facc;
  if (n & 1) {
    hipError_t e = hipMemcpyAsync(scr, user, (size_t)L.g.npts * sizeof(C), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && first)
      e = hipMemcpyAsync(S.facc, aux, (size_t)L.g.face_off[6] * sizeof(double2), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    src = scr;
    dst = user;
    fsrc = S.facc;
    fdst = aux;
  }
  const T* V = static_cast<const T*>(V_v);
  const dim3 g(a.ntiles), b(64 * rows4<T>());
  const bool full = a.nx == kCols;
  for (int s = 0; s < n; ++s) {
    if (L.fused_shell) {
      // the condition-free sweep, then the boundary-shell rounds (new aux,
      // the boundary's correction added to the swept state)
      launch4<T, 0>(tm, full, g, b, st, src, dst, V, a, nullptr, nullptr);
      const hipError_t e = launch_shell_rounds(L, L.shell, src, V_v, fsrc, fdst, dst, st, tm);
      if (e != hipSuccess) return e;
    } else if (L.order == ABC_FIRST) launch4<T, 3>(tm, full, g, b, st, src, dst, V, a, fsrc, fdst);
    else if (L.order == ABC_ZEROTH) launch4<T, 2>(tm, full, g, b, st, src, dst, V, a, nullptr, nullptr);
    else launch4<T, 0>(tm, full, g, b, st, src, dst, V, a, nullptr, nullptr);
    if (tm) tm->end_step();
    std::swap(src, dst);
    std::swap(fsrc, fdst);
  }
  return hipGetLastError();
}

// one step of B orbitals (arrays [B][npts], aux [B][nface]) on the one-pass
// sweep, one launch (blockIdx.y = orbital, V shared)
template <typename T>
hipError_t step4_orbitals(const abc_launch& L1, int B, const void* src, void* dst, const double2* fsrc, double2* fdst,
                          const void* V_v, hipStream_t st, abc_timer* tm) {
  using C = typename cpx<T>::t;
  FusedArgs a = make_args4<T>(L1);
  a.has_V = V_v != nullptr;
  a.bstride = L1.g.npts;
  a.fstride = L1.g.face_off[6];
  const dim3 g(a.ntiles, B), b(64 * rows4<T>());
  const bool full = a.nx == kCols;
  const C* s = static_cast<const C*>(src);
  C* d = static_cast<C*>(dst);
  const T* V = static_cast<const T*>(V_v);
  if (L1.order == ABC_FIRST) launch4<T, 3>(tm, full, g, b, st, s, d, V, a, fsrc, fdst);
  else if (L1.order == ABC_ZEROTH) launch4<T, 2>(tm, full, g, b, st, s, d, V, a, nullptr, nullptr);
  else launch4<T, 0>(tm, full, g, b, st, s, d, V, a, nullptr, nullptr);
  return hipGetLastError();
}

template <typename T>
hipError_t step_t(const abc_launch& L, const abc_scratch& S, void* psi_v, double2* aux, const void* V_v, int n,
                  hipStream_t st, abc_timer* tm) {
  if (L.fused_stages == 4) return step4_t<T>(L, S, psi_v, aux, V_v, n, st, tm);
  using C = typename cpx<T>::t;
  FusedArgs a = make_args<T>(L);
  a.has_V = V_v != nullptr;
  C* user = static_cast<C*>(psi_v);
  C* scr = static_cast<C*>(S.y[0]);
  C* mid = static_cast<C*>(S.y[1]);
  double2* fuser = aux;
  double2* fscr = S.facc;
  double2* vmid = S.g[0];
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
  const int nthreads2 = 64 * (kTY2 + 2 * kHalo2);
  const double dt = L.dt;
  const int tz = L.fused_tz;
  const dim3 g1(a.ntiles), b2(nthreads2);
  const double2* none = nullptr;
  double2* none_w = nullptr;
  for (int s = 0; s < n; ++s) {
    {
      if (L.order == ABC_ZEROTH) {
        launch2<T, 2, true>(tm, "fused2_half_a", tz, g1, b2, st, (const C*)src, (const C*)src, mid, V, a, dt / 4,
                            dt / 3, none, none, none_w, (C*)nullptr);
        launch2<T, 2, false>(tm, "fused2_half_b", tz, g1, b2, st, (const C*)mid, (const C*)src, dst, V, a, dt / 2,
                             dt, none, none, none_w, (C*)nullptr);
      } else if (first) {
        launch2<T, 3, true>(tm, "fused2_half_a", tz, g1, b2, st, (const C*)src, (const C*)src, mid, V, a, dt / 4,
                            dt / 3, (const double2*)fsrc, (const double2*)fsrc, vmid, (C*)nullptr);
        launch2<T, 3, false>(tm, "fused2_half_b", tz, g1, b2, st, (const C*)mid, (const C*)src, dst, V, a, dt / 2,
                             dt, (const double2*)vmid, (const double2*)fsrc, fdst, (C*)nullptr);
      } else {
        launch2<T, 0, true>(tm, "fused2_half_a", tz, g1, b2, st, (const C*)src, (const C*)src, mid, V, a, dt / 4,
                            dt / 3, none, none, none_w, (C*)nullptr);
        launch2<T, 0, false>(tm, "fused2_half_b", tz, g1, b2, st, (const C*)mid, (const C*)src, dst, V, a, dt / 2,
                             dt, none, none, none_w, (C*)nullptr);
      }
    }
    if (tm) tm->end_step();
    std::swap(src, dst);
    std::swap(fsrc, fdst);
  }
  return hipGetLastError();
}

// One step out of place on the two-stage kernels, keeping the Horner
// intermediates u1, u2, u3 of the step (keep[0..2], psi-sized): half A writes
// u2 and keeps its stage-1 output u3, half B keeps u1.
template <typename T>
hipError_t step_keep_t(const abc_launch& L, const abc_scratch& S, const void* psi_in, const double2* aux_in,
                       void* psi_out, double2* aux_out, const void* V_v, void* const* keep, hipStream_t st) {
  using C = typename cpx<T>::t;
  FusedArgs a = make_args<T>(L);
  a.has_V = V_v != nullptr;
  const C* src = static_cast<const C*>(psi_in);
  C* dst = static_cast<C*>(psi_out);
  C* u1 = static_cast<C*>(keep[0]);
  C* u2 = static_cast<C*>(keep[1]);
  C* u3 = static_cast<C*>(keep[2]);
  const T* V = static_cast<const T*>(V_v);
  const double dt = L.dt;
  const int tz = L.fused_tz;
  const dim3 g1(a.ntiles), b2(64 * (kTY2 + 2 * kHalo2));
  const double2* none = nullptr;
  double2* none_w = nullptr;
  double2* vmid = S.g[0];
  if (L.order == ABC_ZEROTH) {
    launch2<T, 2, true>(nullptr, "", tz, g1, b2, st, src, src, u2, V, a, dt / 4, dt / 3, none, none, none_w, u3);
    launch2<T, 2, false>(nullptr, "", tz, g1, b2, st, (const C*)u2, src, dst, V, a, dt / 2, dt, none, none, none_w,
                         u1);
  } else if (L.order == ABC_FIRST) {
    launch2<T, 3, true>(nullptr, "", tz, g1, b2, st, src, src, u2, V, a, dt / 4, dt / 3, aux_in, aux_in, vmid, u3);
    launch2<T, 3, false>(nullptr, "", tz, g1, b2, st, (const C*)u2, src, dst, V, a, dt / 2, dt,
                         (const double2*)vmid, aux_in, aux_out, u1);
  } else {
    launch2<T, 0, true>(nullptr, "", tz, g1, b2, st, src, src, u2, V, a, dt / 4, dt / 3, none, none, none_w, u3);
    launch2<T, 0, false>(nullptr, "", tz, g1, b2, st, (const C*)u2, src, dst, V, a, dt / 2, dt, none, none, none_w,
                         u1);
  }
  return hipGetLastError();
}

// The same keeping the increments: keep[2] = u3 - z, keep[1] = u2 - z,
// keep[0] = u1 - z (z the step's input); u2 itself goes to S.y[1].
template <typename T>
hipError_t step_keepd_t(const abc_launch& L, const abc_scratch& S, const void* psi_in, const double2* aux_in,
                        void* psi_out, double2* aux_out, const void* V_v, void* const* keep, hipStream_t st) {
  using C = typename cpx<T>::t;
  FusedArgs a = make_args<T>(L);
  a.has_V = V_v != nullptr;
  const C* src = static_cast<const C*>(psi_in);
  C* dst = static_cast<C*>(psi_out);
  C* mid = static_cast<C*>(S.y[1]);
  C* d1 = static_cast<C*>(keep[0]);
  C* d2 = static_cast<C*>(keep[1]);
  C* d3 = static_cast<C*>(keep[2]);
  const T* V = static_cast<const T*>(V_v);
  const double dt = L.dt;
  const int tz = L.fused_tz;
  const dim3 g1(a.ntiles), b2(64 * (kTY2 + 2 * kHalo2));
  const double2* none = nullptr;
  double2* none_w = nullptr;
  double2* vmid = S.g[0];
  C* nul = nullptr;
  if (L.order == ABC_ZEROTH) {
    launch2_keepd<T, 2, true>(tz, g1, b2, st, src, src, mid, V, a, dt / 4, dt / 3, none, none, none_w, d3, d2);
    launch2_keepd<T, 2, false>(tz, g1, b2, st, (const C*)mid, src, dst, V, a, dt / 2, dt, none, none, none_w, d1,
                               nul);
  } else if (L.order == ABC_FIRST) {
    launch2_keepd<T, 3, true>(tz, g1, b2, st, src, src, mid, V, a, dt / 4, dt / 3, aux_in, aux_in, vmid, d3, d2);
    launch2_keepd<T, 3, false>(tz, g1, b2, st, (const C*)mid, src, dst, V, a, dt / 2, dt, (const double2*)vmid,
                               aux_in, aux_out, d1, nul);
  } else {
    launch2_keepd<T, 0, true>(tz, g1, b2, st, src, src, mid, V, a, dt / 4, dt / 3, none, none, none_w, d3, d2);
    launch2_keepd<T, 0, false>(tz, g1, b2, st, (const C*)mid, src, dst, V, a, dt / 2, dt, none, none, none_w, d1,
                               nul);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step_fused_keepd(const abc_launch& L, const abc_scratch& S, const void* psi_in,
                                   const double2* aux_in, void* psi_out, double2* aux_out, const void* V,
                                   void* const* keep, hipStream_t st) {
  if (L.dtype != ABC_C128) return hipErrorInvalidValue;
  return step_keepd_t<double>(L, S, psi_in, aux_in, psi_out, aux_out, V, keep, st);
}

hipError_t launch_step_fused_keep(const abc_launch& L, const abc_scratch& S, const void* psi_in,
                                  const double2* aux_in, void* psi_out, double2* aux_out, const void* V,
                                  void* const* keep, hipStream_t st) {
  if (L.dtype == ABC_C64) return step_keep_t<float>(L, S, psi_in, aux_in, psi_out, aux_out, V, keep, st);
  return step_keep_t<double>(L, S, psi_in, aux_in, psi_out, aux_out, V, keep, st);
}

hipError_t launch_step_fused(const abc_launch& L, const abc_scratch& S, void* psi, double2* aux, const void* V,
                             int n_steps, hipStream_t st, abc_timer* tm) {
  if (L.dtype == ABC_C64) return step_t<float>(L, S, psi, aux, V, n_steps, st, tm);
  return step_t<double>(L, S, psi, aux, V, n_steps, st, tm);
}

// ---------------------------------------------------------------------------
// Batched boxes: one descriptor-driven launch per half-step for every group of
// boxes that share (order, precision, tile depth).
// ---------------------------------------------------------------------------

size_t fused_batch_desc_bytes(int nbox) { return (size_t)4 * nbox * sizeof(Box2); }

int fused_batch_build(const std::vector<FusedMember>& m, void* host, int n) {
  const int nb = (int)m.size();
  Box2* hb = static_cast<Box2*>(host);
  int total = 0;
  // descriptor sets [parity][half]; each box keeps its own ping-pong, arranged
  // like the single-box path so that the last step writes the caller's buffers
  for (int i = 0; i < nb; ++i) {
    const abc_launch& L = *m[i].L;
    const abc_scratch& S = *m[i].S;
    FusedArgs a = L.dtype == ABC_C64 ? make_args<float>(L) : make_args<double>(L);
    a.has_V = m[i].V != nullptr;
    char* user = static_cast<char*>(m[i].psi);
    char* scr = static_cast<char*>(S.y[0]);
    char* mid = static_cast<char*>(S.y[1]);
    double2* fuser = m[i].aux;
    double2* fscr = S.facc;
    double2* vmid = S.g[0];
    const bool first = L.order == ABC_FIRST;
    char* src0 = (n & 1) ? scr : user;
    char* dst0 = (n & 1) ? user : scr;
    double2* fsrc0 = (n & 1) ? fscr : fuser;
    double2* fdst0 = (n & 1) ? fuser : fscr;
    for (int q = 0; q < 2; ++q) {
      char* src = q == 0 ? src0 : dst0;
      char* dst = q == 0 ? dst0 : src0;
      double2* fsrc = q == 0 ? fsrc0 : fdst0;
      double2* fdst = q == 0 ? fdst0 : fsrc0;
      Box2& A = hb[(q * 2 + 0) * nb + i];
      Box2& B = hb[(q * 2 + 1) * nb + i];
      A.a = a;
      A.w = src;
      A.base = src;
      A.out = mid;
      A.V = m[i].V;
      A.av = first ? fsrc : nullptr;
      A.fb = first ? fsrc : nullptr;
      A.aux_out = first ? vmid : nullptr;
      A.tile_begin = total;
      A.pad = 0;
      B = A;
      B.w = mid;
      B.av = first ? vmid : nullptr;
      B.out = dst;
      B.aux_out = first ? fdst : nullptr;
    }
    total += a.ntiles;
  }
  return total;
}

hipError_t launch_batch_fused(const std::vector<FusedMember>& m, int tz, const void* dev, int total, int n,
                              hipStream_t st, abc_timer* tm) {
  const int nb = (int)m.size();
  if (nb == 0 || n <= 0) return hipSuccess;
  const abc_launch& L0 = *m[0].L;
  // the descriptors' tile counts come from each box's depth; the kernels are
  // instantiated at tz, so every box must have been built at that depth
  for (int i = 0; i < nb; ++i)
    if (m[i].L->fused_tz != tz) return hipErrorInvalidValue;
  if (n & 1)
    for (int i = 0; i < nb; ++i) {
      const abc_launch& L = *m[i].L;
      const size_t csz = L.dtype == ABC_C64 ? 8 : 16;
      hipError_t e = hipMemcpyAsync(m[i].S->y[0], m[i].psi, (size_t)L.g.npts * csz, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess && L.order == ABC_FIRST)
        e = hipMemcpyAsync(m[i].S->facc, m[i].aux, (size_t)L.g.face_off[6] * sizeof(double2),
                           hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return e;
    }
  const Box2* db = static_cast<const Box2*>(dev);
  const dim3 g((unsigned)((total + 7) / 8 * 8));
  const int order = L0.order;
  const bool c64 = L0.dtype == ABC_C64;
  for (int s = 0; s < n; ++s) {
    const int q = s & 1;
    const Box2* dA = db + (q * 2 + 0) * nb;
    const Box2* dB = db + (q * 2 + 1) * nb;
#define ABC_BATCH_PAIR(T, ORD)                                                        \
  do {                                                                                \
    launch2_batch<T, ORD, true>(tm, "fused2_batch_a", tz, g, st, dA, nb, total, 0);   \
    launch2_batch<T, ORD, false>(tm, "fused2_batch_b", tz, g, st, dB, nb, total, 1);  \
  } while (0)
    if (c64) {
      if (order == ABC_FIRST) ABC_BATCH_PAIR(float, 3);
      else if (order == ABC_ZEROTH) ABC_BATCH_PAIR(float, 2);
      else ABC_BATCH_PAIR(float, 0);
    } else {
      if (order == ABC_FIRST) ABC_BATCH_PAIR(double, 3);
      else if (order == ABC_ZEROTH) ABC_BATCH_PAIR(double, 2);
      else ABC_BATCH_PAIR(double, 0);
    }
#undef ABC_BATCH_PAIR
    if (tm) tm->end_step();
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Orbital batches on the fused path
// ---------------------------------------------------------------------------
namespace {

// [n][B] <-> [B][n] through an LDS tile of 64 rows x B (B <= 64)
template <typename E>
__global__ void __launch_bounds__(256) aos_soa_kernel(const E* __restrict__ in, E* __restrict__ out, long long n,
                                                      int B, int to_soa) {
  extern __shared__ unsigned char smem[];
  E* tile = reinterpret_cast<E*>(smem);  // [B][65]
  const long long i0 = (long long)blockIdx.x * 64;
  const int cnt = (int)min((long long)64, n - i0);
  if (to_soa) {
    for (int t = threadIdx.x; t < cnt * B; t += blockDim.x) {
      const int i = t / B, b = t - i * B;
      tile[b * 65 + i] = in[(i0 + i) * B + b];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 64 * B; t += blockDim.x) {
      const int b = t >> 6, i = t & 63;
      if (i < cnt) out[(long long)b * n + i0 + i] = tile[b * 65 + i];
    }
  } else {
    for (int t = threadIdx.x; t < 64 * B; t += blockDim.x) {
      const int b = t >> 6, i = t & 63;
      if (i < cnt) tile[b * 65 + i] = in[(long long)b * n + i0 + i];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < cnt * B; t += blockDim.x) {
      const int i = t / B, b = t - i * B;
      out[(i0 + i) * B + b] = tile[b * 65 + i];
    }
  }
}

template <typename E>
hipError_t transpose(const void* in, void* out, long long n, int B, bool to_soa, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 63) / 64);
  aos_soa_kernel<E><<<blocks, 256, (size_t)B * 65 * sizeof(E), st>>>(static_cast<const E*>(in), static_cast<E*>(out),
                                                                      n, B, to_soa ? 1 : 0);
  return hipGetLastError();
}

// V + t0 rho + t3 rho^2 with rho = sum_b |psi_b|^2 (Sec. 4.3 mean field,
// simplified functional), from the orbital arrays of the current state
template <typename T>
__global__ void __launch_bounds__(256) meanfield_soa_kernel(const typename cpx<T>::t* __restrict__ cur,
                                                            const T* __restrict__ V, T* __restrict__ veff,
                                                            long long n, int B, T t0, T t3) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  T rho = 0;
  for (int b = 0; b < B; ++b) {
    const auto v = cur[(long long)b * n + p];
    rho += v.x * v.x + v.y * v.y;
  }
  const T base = V ? V[p] : T(0);
  veff[p] = base + t0 * rho + t3 * rho * rho;
}

// one step of parity q over every box of a batch (descriptors already on the
// device, ping-pong arranged by fused_batch_build)
hipError_t launch_batch_step(const abc_launch& L0, int nb, int tz, const void* dev, int total, int q,
                             hipStream_t st, abc_timer* tm) {
  const Box2* db = static_cast<const Box2*>(dev);
  const dim3 g((unsigned)((total + 7) / 8 * 8));
  const Box2* dA = db + (q * 2 + 0) * nb;
  const Box2* dB = db + (q * 2 + 1) * nb;
  const int order = L0.order;
#define ABC_BATCH_PAIR(T, ORD)                                                        \
  do {                                                                                \
    launch2_batch<T, ORD, true>(tm, "fused2_batch_a", tz, g, st, dA, nb, total, 0);   \
    launch2_batch<T, ORD, false>(tm, "fused2_batch_b", tz, g, st, dB, nb, total, 1);  \
  } while (0)
  if (L0.dtype == ABC_C64) {
    if (order == ABC_FIRST) ABC_BATCH_PAIR(float, 3);
    else if (order == ABC_ZEROTH) ABC_BATCH_PAIR(float, 2);
    else ABC_BATCH_PAIR(float, 0);
  } else {
    if (order == ABC_FIRST) ABC_BATCH_PAIR(double, 3);
    else if (order == ABC_ZEROTH) ABC_BATCH_PAIR(double, 2);
    else ABC_BATCH_PAIR(double, 0);
  }
#undef ABC_BATCH_PAIR
  return hipGetLastError();
}

}  // namespace

size_t orbital_batch_bytes(const abc_launch& L1, int B, bool first, bool meanfield) {
  const size_t csz = L1.dtype == ABC_C64 ? 8 : 16, rsz = L1.dtype == ABC_C64 ? 4 : 8;
  return 3 * (size_t)B * L1.g.npts * csz + (first ? 3 * (size_t)B * L1.g.face_off[6] * 16 : 0) +
         (meanfield ? (size_t)L1.g.npts * rsz : 0) + 2 * fused_batch_desc_bytes(B);
}

hipError_t launch_step_orbitals(OrbitalBatch& ob, void* psi, double2* aux, const void* V, int n, hipStream_t st,
                                abc_timer* tm) {
  if (n <= 0) return hipSuccess;
  const abc_launch& L1 = ob.L1;
  const int B = ob.B;
  const long long np = L1.g.npts, nf = L1.g.face_off[6];
  const bool c64 = L1.dtype == ABC_C64;
  const bool first = L1.order == ABC_FIRST;
  const size_t csz = c64 ? 8 : 16;
  // the initial state goes where fused_batch_build expects it (array B for
  // an odd count), so that the result ends in array A
  const int in = (n & 1) ? 1 : 0;
  hipError_t e = c64 ? transpose<float2>(psi, ob.soa[in], np, B, true, st)
                     : transpose<double2>(psi, ob.soa[in], np, B, true, st);
  if (e == hipSuccess && first) e = transpose<double2>(aux, ob.soa_f[in], nf, B, true, st);
  if (e != hipSuccess) return e;
  std::vector<FusedMember> m(B);
  for (int b = 0; b < B; ++b) {
    abc_scratch& S = ob.S[b];
    S.y[0] = static_cast<char*>(ob.soa[1]) + (size_t)b * np * csz;
    S.y[1] = static_cast<char*>(ob.soa[2]) + (size_t)b * np * csz;
    if (first) {
      S.facc = ob.soa_f[1] + (size_t)b * nf;
      S.g[0] = ob.soa_f[2] + (size_t)b * nf;
    }
    m[b] = {&L1, &S, static_cast<char*>(ob.soa[0]) + (size_t)b * np * csz, first ? ob.soa_f[0] + (size_t)b * nf : nullptr,
            ob.veff ? ob.veff : V};
  }
  if (L1.fused_stages == 4) {
    // one-pass sweep over all orbitals in one launch per step (blockIdx.y =
    // orbital); the ping-pong between arrays A and B ends in A
    for (int s = 0; s < n; ++s) {
      const int cur = (s & 1) == 0 ? in : 1 - in;
      if (ob.veff) {
        const void* cs = ob.soa[cur];
        const unsigned blocks = (unsigned)((np + 255) / 256);
        if (L1.meanfield == ABC_MF_SKYRME)
          e = skyrme_veff(*L1.pot, cs, true, B, c64, V, ob.veff, L1.t0, L1.t3, st, tm);
        else if (c64)
          abc_launch_kernel(tm, "meanfield", meanfield_soa_kernel<float>, dim3(blocks), dim3(256), st,
                            static_cast<const float2*>(cs), static_cast<const float*>(V),
                            static_cast<float*>(ob.veff), np, B, float(L1.t0), float(L1.t3));
        else
          abc_launch_kernel(tm, "meanfield", meanfield_soa_kernel<double>, dim3(blocks), dim3(256), st,
                            static_cast<const double2*>(cs), static_cast<const double*>(V),
                            static_cast<double*>(ob.veff), np, B, L1.t0, L1.t3);
        if (e != hipSuccess) return e;
      }
      const void* Vs = ob.veff ? ob.veff : V;
      e = c64 ? step4_orbitals<float>(L1, B, ob.soa[cur], ob.soa[1 - cur], first ? ob.soa_f[cur] : nullptr,
                                      first ? ob.soa_f[1 - cur] : nullptr, Vs, st, tm)
              : step4_orbitals<double>(L1, B, ob.soa[cur], ob.soa[1 - cur], first ? ob.soa_f[cur] : nullptr,
                                       first ? ob.soa_f[1 - cur] : nullptr, Vs, st, tm);
      if (e != hipSuccess) return e;
      if (tm) tm->end_step();
    }
    e = c64 ? transpose<float2>(ob.soa[0], psi, np, B, false, st) : transpose<double2>(ob.soa[0], psi, np, B, false, st);
    if (e == hipSuccess && first) e = transpose<double2>(ob.soa_f[0], aux, nf, B, false, st);
    return e;
  }
  const int par = n & 1;
  const size_t dbytes = fused_batch_desc_bytes(B);
  const void* vkey = ob.veff ? ob.veff : V;
  const void* ddev = static_cast<char*>(ob.desc_dev) + par * dbytes;
  if (!ob.desc_ok[par] || ob.desc_V[par] != vkey) {
    // a new descriptor set: never inside a graph capture (the copy would
    // read host memory that a later call may rewrite)
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
      return hipErrorStreamCaptureUnsupported;
    if (ob.pending && hipEventSynchronize(ob.copied) != hipSuccess) return hipErrorUnknown;
    void* dhost = static_cast<char*>(ob.desc_host) + par * dbytes;
    ob.desc_total = fused_batch_build(m, dhost, n);
    e = hipMemcpyAsync(const_cast<void*>(ddev), dhost, dbytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(ob.copied, st);
    if (e != hipSuccess) return e;
    ob.pending = true;
    ob.desc_V[par] = vkey;
    ob.desc_ok[par] = true;
  }
  const int total = ob.desc_total;
  for (int s = 0; s < n; ++s) {
    const int q = s & 1;
    if (ob.veff) {
      // the current state: array `in` for even s, the other one for odd s
      const void* cur = ob.soa[q == 0 ? in : 1 - in];
      const unsigned blocks = (unsigned)((np + 255) / 256);
      if (L1.meanfield == ABC_MF_SKYRME)
        e = skyrme_veff(*L1.pot, cur, true, B, c64, V, ob.veff, L1.t0, L1.t3, st, tm);
      else if (c64)
        abc_launch_kernel(tm, "meanfield", meanfield_soa_kernel<float>, dim3(blocks), dim3(256), st,
                          static_cast<const float2*>(cur), static_cast<const float*>(V), static_cast<float*>(ob.veff),
                          np, B, float(L1.t0), float(L1.t3));
      else
        abc_launch_kernel(tm, "meanfield", meanfield_soa_kernel<double>, dim3(blocks), dim3(256), st,
                          static_cast<const double2*>(cur), static_cast<const double*>(V),
                          static_cast<double*>(ob.veff), np, B, L1.t0, L1.t3);
      if (e != hipSuccess) return e;
    }
    e = launch_batch_step(L1, B, ob.tz, ddev, total, q, st, tm);
    if (e != hipSuccess) return e;
    if (tm) tm->end_step();
  }
  e = c64 ? transpose<float2>(ob.soa[0], psi, np, B, false, st) : transpose<double2>(ob.soa[0], psi, np, B, false, st);
  if (e == hipSuccess && first) e = transpose<double2>(ob.soa_f[0], aux, nf, B, false, st);
  return e;
}
