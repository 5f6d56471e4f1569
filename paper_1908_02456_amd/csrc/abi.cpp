// C ABI of libabc_dtn: parameter checks, operator setup and upload, scratch
// ownership and dispatch of the device paths.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <rocblas/rocblas.h>

#include "abc_internal.h"
#include "fused.h"

namespace {

thread_local std::string g_last_error;

abc_status fail(abc_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

}  // namespace

struct abc_ctx {
  abc_params p{};
  abc_launch L{};
  abc_scratch S{};
  abc::FaceOps face;
  std::vector<void*> allocations;
  size_t bytes = 0;
  size_t aux_elems = 0;
  int n_gamma = 0;
  int box_rank = 0;         // box form: dimension the second order interpolates in
  double box_bound = 0;    // box form: spectral bound of the boundary block
  int use_fused = 0;
  double2* box_mat = nullptr;
  double2* box_q = nullptr;
  std::vector<std::string> launch_labels;  // launches of a step, from the last abc_step_timed
  OrbitalBatch* orb = nullptr;             // fused path over an orbital batch / mean field
  abc_launch La{};                         // adjoint operator set (built on first abc_adjoint)
  bool adjoint_ready = false;
  PotentialSolver pot;                     // ABC_MF_SKYRME solves
  FaceFFT fft{};                           // exact face sections by FFT
  long long mon_steps = 0;                 // steps taken by abc_step_monitored
  long long mon_records = 0;               // records it has written
  double* mon_prevW = nullptr;             // W of the last record, per orbital
};

namespace {

abc_status dev_alloc(abc_ctx* c, void** ptr, size_t bytes) {
  if (bytes == 0) {
    *ptr = nullptr;
    return ABC_OK;
  }
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) return fail(ABC_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  c->allocations.push_back(*ptr);
  c->bytes += bytes;
  return ABC_OK;
}

abc_status check_params(const abc_params& p) {
  if (p.nx < 1 || p.ny < 1 || p.nz < 1) return fail(ABC_EINVAL, "box sizes must be positive");
  if (p.radius < 1 || p.radius > abc::kMaxR) return fail(ABC_EINVAL, "radius must be 1, 2 or 3");
  if (p.nx < 2 * p.radius + 1 || p.ny < 2 * p.radius + 1 || p.nz < 2 * p.radius + 1)
    return fail(ABC_EINVAL, "every axis needs at least 2R+1 points");
  if (!(p.h > 0) || !(p.dt > 0) || !std::isfinite(p.h) || !std::isfinite(p.dt))
    return fail(ABC_EINVAL, "h and dt must be positive and finite");
  if (p.order < ABC_DIRICHLET || p.order > ABC_SECOND) return fail(ABC_EINVAL, "unknown order");
  if (p.form != ABC_FORM_BOX && p.form != ABC_FORM_FACES) return fail(ABC_EINVAL, "unknown form");
  if (p.dtype != ABC_C128 && p.dtype != ABC_C64) return fail(ABC_EINVAL, "unknown dtype");
  if (p.batch < 1) return fail(ABC_EINVAL, "batch must be >= 1");
  if (p.meanfield < ABC_MF_NONE || p.meanfield > ABC_MF_SKYRME) return fail(ABC_EINVAL, "unknown mean field");
  if (p.meanfield == ABC_MF_SKYRME) {
    if (!std::isfinite(p.t0) || !std::isfinite(p.t3) || !std::isfinite(p.v0) || !std::isfinite(p.e2))
      return fail(ABC_EINVAL, "mean field: t0, t3, v0 and e2 must be finite");
    if (p.v0 != 0.0 && !(p.a_yukawa > 0 && std::isfinite(p.a_yukawa)))
      return fail(ABC_EINVAL, "mean field: the Yukawa range must be positive");
    if (!(p.pcg_tol > 0 && std::isfinite(p.pcg_tol)) || p.pcg_maxit < 1)
      return fail(ABC_EINVAL, "mean field: pcg_tol > 0 and pcg_maxit >= 1");
  }
  if (p.pcg_fixed < 0) return fail(ABC_EINVAL, "pcg_fixed must be >= 0");
  for (int i = 0; i < 2; ++i)
    if (p.reserved2[i] != 0) return fail(ABC_EINVAL, "reserved fields must be zero");
  if (p.path < ABC_PATH_AUTO || p.path > ABC_PATH_ONEPASS) return fail(ABC_EINVAL, "unknown path");
  if (p.window < 0) return fail(ABC_EINVAL, "window must be >= 0");
  if (p.order == ABC_PERIODIC && p.nx < 2 * p.radius + 1) return fail(ABC_EINVAL, "periodic box too small");
  if (p.order == ABC_ZEROTH && !(p.s0 > 0)) return fail(ABC_EUNSTABLE, "s0 must be positive (zeroth-order theorem)");
  if (p.order == ABC_FIRST && !(p.s1 > 0)) return fail(ABC_EUNSTABLE, "s1 must be positive (first-order theorem)");
  if (p.order == ABC_FIRST && p.form == ABC_FORM_FACES && p.s2 > 0)
    return fail(ABC_ENOTSUP, "the face form implements the theorem's (s1, infinity) pair only");
  if (p.order == ABC_SECOND) {
    // four-point interpolation (Sec. 3.3): the system is singular unless the
    // points are distinct
    const double sp[4] = {p.s1, p.s2, p.s3, p.s4};
    for (int i = 0; i < 4; ++i) {
      if (!(sp[i] > 0) || !std::isfinite(sp[i])) return fail(ABC_EINVAL, "second order: s1..s4 must be positive");
      for (int j = 0; j < i; ++j)
        if (sp[i] == sp[j]) return fail(ABC_EINVAL, "second order: s1..s4 must be distinct");
    }
    if (p.form != ABC_FORM_BOX)
      return fail(ABC_ENOTSUP, "second order: box form only (the face sections lose stability)");
  }
  if (p.diag_every < 0) return fail(ABC_EINVAL, "diag_every must be >= 0");
  for (int i = 0; i < 2; ++i)
    if (p.reserved[i] != 0) return fail(ABC_EINVAL, "reserved fields must be zero");
  return ABC_OK;
}

}  // namespace

extern "C" {

void abc_params_default(abc_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->nx = p->ny = p->nz = 32;
  p->h = 0.2;
  p->dt = 0.002;
  p->radius = 1;
  p->order = ABC_FIRST;
  p->form = ABC_FORM_FACES;
  p->s0 = 1.0;
  p->s1 = 1.0;
  p->s2 = 0.0;
  p->s3 = 3.0;
  p->s4 = 10.0;
  p->a_yukawa = 1.0;
  p->pcg_tol = 1e-12;
  p->pcg_maxit = 1000;
  p->window = 0;
  p->fejer = 1;
  p->dtype = ABC_C128;
  p->batch = 1;
  p->meanfield = ABC_MF_NONE;
  p->path = ABC_PATH_AUTO;
}

const char* abc_last_error(void) { return g_last_error.c_str(); }

void abc_destroy(abc_ctx* c) {
  if (!c) return;
  if (c->pot.host) (void)hipHostFree(c->pot.host);
  if (c->pot.blas) rocblas_destroy_handle(static_cast<rocblas_handle>(c->pot.blas));
  if (c->orb) {
    if (c->orb->copied) hipEventDestroy(c->orb->copied);
    if (c->orb->desc_host) hipHostFree(c->orb->desc_host);
    delete c->orb;
  }
  for (void* ptr : c->allocations) (void)hipFree(ptr);
  delete c;
}

abc_status abc_setup(const abc_params* pp, abc_ctx** out) {
  g_last_error.clear();
  if (!pp || !out) return fail(ABC_EINVAL, "null argument");
  *out = nullptr;
  abc_status st = check_params(*pp);
  if (st != ABC_OK) return st;
  const abc_params& p = *pp;
  abc_ctx* c = new abc_ctx();
  c->p = p;
  abc_launch& L = c->L;
  L.g = abc::make_geometry(p.nx, p.ny, p.nz, p.radius, p.batch);
  L.h = p.h;
  L.dt = p.dt;
  abc::fd_weights(p.radius, L.c);
  L.order = p.order;
  L.form = p.form;
  L.periodic = p.order == ABC_PERIODIC;
  L.dtype = p.dtype;
  L.w = p.window;
  L.meanfield = p.meanfield;
  L.t0 = p.t0;
  L.t3 = p.t3;
  const bool bc = p.order == ABC_ZEROTH || p.order == ABC_FIRST || p.order == ABC_SECOND;

  // spectral bound of the kinetic part: 3 max_theta sigma_1(theta)
  double smax = 0;
  for (int j = 0; j <= 256; ++j) {
    double th = M_PI * j / 256, acc = -L.c[0];
    for (int k = 1; k <= p.radius; ++k) acc -= 2 * L.c[k] * std::cos(k * th);
    smax = std::max(smax, acc / (2 * p.h * p.h));
  }
  double rho = 3 * smax;

  std::string err;
  if (bc && p.form == ABC_FORM_FACES) {
    st = abc::build_face_ops(p, c->face, err);
    if (st != ABC_OK) { abc_destroy(c); return fail(st, err); }
    const int R = p.radius;
    for (int i = 0; i < R * R; ++i) {
      L.a_loc[i] = make_double2(c->face.a[i].real(), c->face.a[i].imag());
      L.q_loc[i] = make_double2(c->face.q[i].real(), c->face.q[i].imag());
    }
    void* kd = nullptr;
    const size_t kb = c->face.kernel.size() * sizeof(double2);
    if ((st = dev_alloc(c, &kd, kb)) != ABC_OK) { abc_destroy(c); return st; }
    if (hipMemcpy(kd, c->face.kernel.data(), kb, hipMemcpyHostToDevice) != hipSuccess) {
      abc_destroy(c);
      return fail(ABC_EDEVICE, "hipMemcpy of face kernel failed");
    }
    L.face_ker = static_cast<const double2*>(kd);
    L.fused_m0 = L.fused_b0 = make_double2(c->face.kernel[0].real(), c->face.kernel[0].imag());
    // exact sections (no taper, window covering every face): apply them by
    // zero-padded 2D FFTs instead of the direct convolution
    if (p.fejer == 0 && p.window >= std::max({p.nx, p.ny, p.nz}) - 1) {
      st = face_fft_setup(L.g, p.radius, p.window, c->face.kernel, c->fft, &c->allocations, &c->bytes, err);
      if (st != ABC_OK) { abc_destroy(c); return fail(st, err); }
      L.face_fft = &c->fft;
    }
    // Lyapunov-weighted block bound: zeroth order adds up to three faces'
    // operators to H; first order couples psi and f through blocks of norm
    // |H_{Gamma,Sigma}| (three faces at a corner) and B acts on f
    if (p.order == ABC_ZEROTH)
      rho += 3 * c->face.symbol_norm;
    else
      rho = std::max(rho, c->face.symbol_norm) + std::sqrt(3.0) * c->face.coupling_norm;
  }
  if (bc && p.form == ABC_FORM_BOX) {
    std::vector<int> glin;
    double bound = 0;
    abc::BoxReduced red;
    st = abc::build_box_ops(p, &c->box_mat, &c->box_q, &c->n_gamma, glin, &bound, &c->box_rank,
                            p.batch == 1 ? &red : nullptr, err);
    c->box_bound = bound;
    if (st != ABC_OK) { abc_destroy(c); return fail(st, err); }
    if (red.red) {
      // one orbital steps the second order in the subspace (the lifted
      // operator stays for the export)
      c->allocations.push_back(red.U);
      c->allocations.push_back(red.Ut);
      c->allocations.push_back(red.red);
      c->bytes += (size_t)2 * c->n_gamma * red.r * 8 + (size_t)6 * red.r * red.r * 16;
      L.box_U = red.U;
      L.box_Ut = red.Ut;
      L.box_red = red.red;
      L.box_r = red.r;
    }
    if (c->box_mat) { c->allocations.push_back(c->box_mat); c->bytes += abc::box_mat_elems(p.order, c->n_gamma) * 16; }
    if (c->box_q) { c->allocations.push_back(c->box_q); c->bytes += (size_t)c->n_gamma * c->n_gamma * 16; }
    L.box_mat = c->box_mat;
    L.box_q = c->box_q;
    L.n_gamma = c->n_gamma;
    std::vector<int> pg(L.g.npts, -1);
    for (int i = 0; i < c->n_gamma; ++i) pg[glin[i]] = i;
    void *gl = nullptr, *pgd = nullptr;
    if ((st = dev_alloc(c, &gl, glin.size() * sizeof(int))) != ABC_OK ||
        (st = dev_alloc(c, &pgd, pg.size() * sizeof(int))) != ABC_OK) {
      abc_destroy(c);
      return st;
    }
    if (hipMemcpy(gl, glin.data(), glin.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(pgd, pg.data(), pg.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
      abc_destroy(c);
      return fail(ABC_EDEVICE, "hipMemcpy of Gamma maps failed");
    }
    L.gamma_lin = static_cast<const int*>(gl);
    L.point_gamma = static_cast<const int*>(pgd);
    // zeroth: M adds to H; first and second: the boundary block (B, or the
    // (f, g) block [[0, I], [B0, B1]]) beside H, coupled through blocks of
    // the size of H_{Gamma,Sigma}
    rho = p.order == ABC_ZEROTH ? rho + bound : std::max(rho, bound) + std::sqrt(3.0) * 2.0 * std::abs(L.c[1]) / (2 * p.h * p.h);
  }
  // fourth-order Taylor polynomial: |T4(i y)| <= 1 requires |y| <= 2 sqrt(2)
  if (p.dt * rho > 2.0 * std::sqrt(2.0)) {
    abc_destroy(c);
    return fail(ABC_EUNSTABLE, "dt times the spectral bound exceeds the Taylor-4 stability limit 2 sqrt(2) (dt * bound = " +
                                   std::to_string(p.dt * rho) + ")");
  }

  // scratch
  const size_t csz = p.dtype == ABC_C64 ? 8 : 16;
  const size_t rsz = p.dtype == ABC_C64 ? 4 : 8;
  const size_t nel = (size_t)L.g.npts * p.batch;
  abc_scratch& S = c->S;
  size_t naux = 0;
  if (bc) naux = p.form == ABC_FORM_BOX ? (size_t)c->n_gamma * p.batch : (size_t)L.g.face_off[6];
  if (p.order == ABC_SECOND) naux *= 2;  // f and g
  c->aux_elems = p.order == ABC_FIRST || p.order == ABC_SECOND ? naux : 0;
  S.red_blocks = 256 + 64;
  void* tmp = nullptr;
  if ((st = dev_alloc(c, &S.y[0], nel * csz)) != ABC_OK || (st = dev_alloc(c, &S.y[1], nel * csz)) != ABC_OK ||
      (st = dev_alloc(c, &S.acc, nel * csz)) != ABC_OK) {
    abc_destroy(c);
    return st;
  }
  if (bc) {
    if ((st = dev_alloc(c, &tmp, naux * 16)) != ABC_OK) { abc_destroy(c); return st; }
    S.g[0] = static_cast<double2*>(tmp);
    if ((st = dev_alloc(c, &tmp, naux * 16)) != ABC_OK) { abc_destroy(c); return st; }
    S.g[1] = static_cast<double2*>(tmp);
    if ((st = dev_alloc(c, &tmp, naux * 16)) != ABC_OK) { abc_destroy(c); return st; }
    S.facc = static_cast<double2*>(tmp);
    if ((st = dev_alloc(c, &tmp, naux * 16)) != ABC_OK) { abc_destroy(c); return st; }
    S.src = static_cast<double2*>(tmp);
    if (p.form == ABC_FORM_BOX && p.batch == 1) {
      // one orbital: E y gathered once per stage for the row-blocked product
      if ((st = dev_alloc(c, &tmp, naux * 16)) != ABC_OK) { abc_destroy(c); return st; }
      S.bwork[0] = static_cast<double2*>(tmp);
      if (L.box_r > 0) {
        // the second order's reduced stages: 6 x n_Gamma packed vectors and
        // 20 r doubles of reduced ones
        if ((st = dev_alloc(c, &tmp, (size_t)6 * c->n_gamma * sizeof(double))) != ABC_OK) { abc_destroy(c); return st; }
        S.bpack = static_cast<double*>(tmp);
        if ((st = dev_alloc(c, &tmp, (size_t)20 * L.box_r * sizeof(double))) != ABC_OK) { abc_destroy(c); return st; }
        S.bred = static_cast<double*>(tmp);
      }
    }
    if (p.form == ABC_FORM_BOX && p.batch > 1) {
      // the operator over the orbital batch is one complex GEMM per stage
      // (the gathered E y and the GEMM result)
      if (p.batch > 64) {
        abc_destroy(c);
        return fail(ABC_ENOTSUP, "box form over an orbital batch: at most 64 orbitals");
      }
      if ((st = dev_alloc(c, &tmp, naux * 16)) != ABC_OK) { abc_destroy(c); return st; }
      S.bwork[0] = static_cast<double2*>(tmp);
      if ((st = dev_alloc(c, &tmp, naux * 16)) != ABC_OK) { abc_destroy(c); return st; }
      S.bwork[1] = static_cast<double2*>(tmp);
      // partial products of the GEMM when its K is split over workgroups
      // (the result has rows x orbitals = naux elements for every order)
      if ((st = dev_alloc(c, &tmp, box_gemm_part_elems(naux) * 16)) != ABC_OK) { abc_destroy(c); return st; }
      S.bpart = static_cast<double2*>(tmp);
    }
  }
  if (p.meanfield) {
    if ((st = dev_alloc(c, &S.veff, (size_t)L.g.npts * rsz)) != ABC_OK) { abc_destroy(c); return st; }
  }
  if ((st = dev_alloc(c, &tmp, (size_t)p.batch * S.red_blocks * 4 * sizeof(double))) != ABC_OK) {
    abc_destroy(c);
    return st;
  }
  S.red = static_cast<double*>(tmp);

  if (p.meanfield == ABC_MF_SKYRME) {
    PotentialSolver& ps = c->pot;
    ps.nx = p.nx;
    ps.ny = p.ny;
    ps.nz = p.nz;
    ps.R = p.radius;
    ps.h = p.h;
    for (int k = 0; k <= abc::kMaxR; ++k) ps.c[k] = L.c[k];
    ps.v0 = p.v0;
    ps.a = p.a_yukawa;
    ps.e2 = p.e2;
    ps.tol = p.pcg_tol;
    ps.maxit = p.pcg_maxit;
    ps.fixed = p.pcg_fixed;
    const size_t np = (size_t)L.g.npts;
    ps.nblk = (int)std::min<size_t>(1024, (np + 255) / 256);
    double** vec[9] = {&ps.rho, &ps.wy, &ps.wc, &ps.r, &ps.p, &ps.q, &ps.t1, &ps.t2, &ps.z};
    for (int i = 0; i < 9 && st == ABC_OK; ++i) {
      st = dev_alloc(c, &tmp, np * sizeof(double));
      *vec[i] = static_cast<double*>(tmp);
    }
    // sine transforms and R = 1 eigenvalues per axis (preconditioner)
    const int dims[3] = {p.nx, p.ny, p.nz};
    double** mats[3] = {&ps.sx, &ps.sy, &ps.sz};
    double** eigs[3] = {&ps.ex, &ps.ey, &ps.ez};
    for (int a = 0; a < 3 && st == ABC_OK; ++a) {
      const int n = dims[a];
      std::vector<double> S((size_t)n * n), ev(n);
      for (int j = 0; j < n; ++j) {
        ev[j] = (2.0 - 2.0 * std::cos(M_PI * (j + 1) / (n + 1))) / (p.h * p.h);
        for (int k = 0; k < n; ++k) S[(size_t)j * n + k] = std::sin(M_PI * (double)(j + 1) * (k + 1) / (n + 1));
      }
      st = dev_alloc(c, &tmp, S.size() * sizeof(double));
      *mats[a] = static_cast<double*>(tmp);
      if (st == ABC_OK) st = dev_alloc(c, &tmp, ev.size() * sizeof(double));
      if (st == ABC_OK) *eigs[a] = static_cast<double*>(tmp);
      if (st == ABC_OK && (hipMemcpy(*mats[a], S.data(), S.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
                           hipMemcpy(*eigs[a], ev.data(), ev.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess))
        st = fail(ABC_EDEVICE, "hipMemcpy failed");
    }
    if (st == ABC_OK) {
      rocblas_handle hb = nullptr;
      if (rocblas_create_handle(&hb) != rocblas_status_success) st = fail(ABC_EDEVICE, "rocblas_create_handle failed");
      else ps.blas = hb;
    }
    if (st == ABC_OK && potential_warmup(ps) != hipSuccess) st = fail(ABC_EDEVICE, "potential solver set-up failed");
    if (st == ABC_OK) st = dev_alloc(c, &tmp, 3 * (size_t)ps.nblk * sizeof(double));
    ps.part = static_cast<double*>(tmp);
    if (st == ABC_OK) st = dev_alloc(c, &tmp, 8 * sizeof(double));
    ps.scal = static_cast<double*>(tmp);
    if (st == ABC_OK) st = dev_alloc(c, &tmp, 3 * sizeof(double));
    ps.tally = static_cast<double*>(tmp);
    if (st == ABC_OK && hipMemset(ps.tally, 0, 3 * sizeof(double)) != hipSuccess)
      st = fail(ABC_EDEVICE, "hipMemset failed");
    if (st == ABC_OK && hipHostMalloc(&tmp, 2 * sizeof(double)) != hipSuccess) st = fail(ABC_ENOMEM, "pinned memory");
    if (st == ABC_OK) ps.host = static_cast<double*>(tmp);
    // the potentials start at zero (the first solve starts from zero)
    if (st == ABC_OK && (hipMemset(ps.wy, 0, np * sizeof(double)) != hipSuccess ||
                         hipMemset(ps.wc, 0, np * sizeof(double)) != hipSuccess ||
                         hipDeviceSynchronize() != hipSuccess))
      st = fail(ABC_EDEVICE, "hipMemset failed");
    if (st != ABC_OK) { abc_destroy(c); return st; }
    L.pot = &ps;
  }

  c->use_fused = 0;
  if (p.path != ABC_PATH_STAGED) {
    std::string why;
    const bool ok = p.path == ABC_PATH_ONEPASS ? fused4_supported(p, &why) : fused_supported(p, &why);
    if ((p.path == ABC_PATH_FUSED || p.path == ABC_PATH_ONEPASS) && !ok) {
      abc_destroy(c);
      return fail(ABC_ENOTSUP, "fused path: " + why);
    }
    c->use_fused = ok ? 1 : 0;
    if (c->use_fused) {
      st = fused_prepare(c->p, c->L, &c->allocations, &c->bytes, err);
      if (st != ABC_OK) { abc_destroy(c); return fail(st, err); }
    }
    if (c->use_fused && (p.batch > 1 || p.meanfield != ABC_MF_NONE)) {
      // orbitals stepped as boxes of one descriptor-driven launch
      c->orb = new OrbitalBatch();
      OrbitalBatch& ob = *c->orb;
      ob.L1 = L;
      ob.L1.g = abc::make_geometry(p.nx, p.ny, p.nz, p.radius, 1);
      ob.B = p.batch;
      ob.tz = L.fused_tz;
      ob.S.assign(p.batch, abc_scratch{});
      const bool first = p.order == ABC_FIRST;
      const size_t np = (size_t)L.g.npts, nf = (size_t)ob.L1.g.face_off[6];
      for (int i = 0; i < 3 && st == ABC_OK; ++i) {
        st = dev_alloc(c, &ob.soa[i], (size_t)p.batch * np * csz);
        if (st == ABC_OK && first) {
          st = dev_alloc(c, &tmp, (size_t)p.batch * nf * 16);
          ob.soa_f[i] = static_cast<double2*>(tmp);
        }
      }
      if (st == ABC_OK && p.meanfield) st = dev_alloc(c, &ob.veff, np * rsz);
      if (st == ABC_OK) st = dev_alloc(c, &ob.desc_dev, 2 * fused_batch_desc_bytes(p.batch));
      if (st == ABC_OK && (hipHostMalloc(&ob.desc_host, 2 * fused_batch_desc_bytes(p.batch)) != hipSuccess ||
                           hipEventCreate(&ob.copied) != hipSuccess))
        st = fail(ABC_ENOMEM, "orbital batch descriptors");
      if (st != ABC_OK) { abc_destroy(c); return st; }
    }
  }
  *out = c;
  return ABC_OK;
}

size_t abc_aux_elems(const abc_ctx* c) { return c ? c->aux_elems : 0; }

size_t abc_device_bytes(const abc_ctx* c) { return c ? c->bytes : 0; }

int abc_path(const abc_ctx* c) {
  if (!c || !c->use_fused) return ABC_PATH_STAGED;
  return c->L.fused_stages == 4 ? ABC_PATH_ONEPASS : ABC_PATH_FUSED;
}

abc_status abc_step(abc_ctx* c, void* psi, void* aux, const void* V, int n_steps, void* stream) {
  if (!c || !psi) return fail(ABC_EINVAL, "null context or psi");
  if (n_steps < 0) return fail(ABC_EINVAL, "n_steps must be >= 0");
  if (c->aux_elems && !aux) return fail(ABC_EINVAL, "first and second order need the aux buffer");
  if (n_steps == 0) return ABC_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
      if (c->p.meanfield == ABC_MF_SKYRME && c->pot.fixed == 0)
        return fail(ABC_EINVAL, "graph capture of an ABC_MF_SKYRME step needs pcg_fixed >= 1 (the adaptive solves "
                                "read their convergence flag on the host)");
      if (c->orb && c->L.fused_stages == 2) {
        const OrbitalBatch& ob = *c->orb;
        const int par = n_steps & 1;
        if (!ob.desc_ok[par] || ob.desc_V[par] != (ob.veff ? ob.veff : V))
          return fail(ABC_EINVAL, "graph capture of an orbital batch: step once outside the capture with the same V "
                                  "and the same parity of n_steps first (the launch descriptors are built then)");
      }
    }
  }
  hipError_t e;
  if (c->orb)
    e = launch_step_orbitals(*c->orb, psi, static_cast<double2*>(aux), V, n_steps, st, nullptr);
  else if (c->use_fused)
    e = launch_step_fused(c->L, c->S, psi, static_cast<double2*>(aux), V, n_steps, st);
  else
    e = launch_step_staged(c->L, c->S, psi, static_cast<double2*>(aux), V, n_steps, st);
  if (e != hipSuccess) return fail(ABC_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return ABC_OK;
}

abc_status abc_step_monitored(abc_ctx* c, void* psi, void* aux, const void* V, int n_steps, void* stream,
                              double* ring, int ring_len, unsigned* flags) {
  if (!c || !psi || !ring || !flags) return fail(ABC_EINVAL, "null argument");
  if (c->p.diag_every < 1) return fail(ABC_EINVAL, "abc_step_monitored: the context's diag_every must be >= 1");
  if (ring_len < 1) return fail(ABC_EINVAL, "abc_step_monitored: ring_len must be >= 1");
  if (n_steps < 0) return fail(ABC_EINVAL, "n_steps must be >= 0");
  if (c->aux_elems && !aux) return fail(ABC_EINVAL, "first and second order need the aux buffer");
  const int B = c->p.batch;
  if (!c->mon_prevW) {
    void* ptr = nullptr;
    abc_status s = dev_alloc(c, &ptr, sizeof(double) * B);
    if (s != ABC_OK) return s;
    c->mon_prevW = static_cast<double*>(ptr);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  // W is non-increasing for every order but the second (Sec. 3); an FP32
  // state carries rounding noise of about 1e-7 in it
  const bool check_w = c->p.order != ABC_SECOND;
  const double tol = c->p.dtype == ABC_C64 ? 1e-6 : 1e-12;
  const size_t rec_len = 3 * (size_t)B + 2;
  const int every = c->p.diag_every;
  int left = n_steps;
  while (left > 0) {
    const int k = std::min<long long>(left, every - c->mon_steps % every);
    abc_status s = abc_step(c, psi, aux, V, k, stream);
    if (s != ABC_OK) return s;
    c->mon_steps += k;
    left -= k;
    if (c->mon_steps % every != 0) continue;
    double* rec = ring + (size_t)(c->mon_records % ring_len) * rec_len;
    hipError_t e = launch_diagnostics(c->L, c->S, psi, static_cast<const double2*>(aux), V, rec + 1, st);
    if (e == hipSuccess)
      e = launch_monitor_check(rec, B, c->mon_steps, c->mon_prevW, c->mon_records > 0, check_w, tol, flags, st);
    if (e != hipSuccess) return fail(ABC_EDEVICE, std::string("monitor launch: ") + hipGetErrorString(e));
    ++c->mon_records;
  }
  return ABC_OK;
}

abc_status abc_step_timed(abc_ctx* c, void* psi, void* aux, const void* V, int n_steps, void* stream, double* ms,
                          int cap, int* launches) {
  if (!c || !psi || !launches || (cap > 0 && !ms)) return fail(ABC_EINVAL, "null argument");
  if (n_steps < 1) return fail(ABC_EINVAL, "n_steps must be >= 1");
  if (c->aux_elems && !aux) return fail(ABC_EINVAL, "first and second order need the aux buffer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  abc_timer tm;
  hipError_t e;
  if (c->orb)
    e = launch_step_orbitals(*c->orb, psi, static_cast<double2*>(aux), V, n_steps, st, &tm);
  else if (c->use_fused)
    e = launch_step_fused(c->L, c->S, psi, static_cast<double2*>(aux), V, n_steps, st, &tm);
  else
    e = launch_step_staged(c->L, c->S, psi, static_cast<double2*>(aux), V, n_steps, st, &tm);
  if (e == hipSuccess) e = tm.err;
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  const int k = (int)tm.labels.size();
  const bool whole = e == hipSuccess && tm.ev.size() == (size_t)n_steps * k;
  if (whole) {
    for (int j = 0; j < cap && j < k; ++j) ms[j] = 0;
    for (size_t i = 0; i < tm.ev.size() && e == hipSuccess; ++i) {
      float t = 0;
      e = hipEventElapsedTime(&t, tm.ev[i].start, tm.ev[i].stop);
      const int j = (int)(i % k);
      if (j < cap) ms[j] += (double)t / n_steps;
    }
  }
  if (e != hipSuccess) return fail(ABC_EDEVICE, std::string("timed step: ") + hipGetErrorString(e));
  if (!whole) return fail(ABC_EDEVICE, "timed step: event count mismatch");
  c->launch_labels = tm.labels;
  *launches = k;
  return ABC_OK;
}

const char* abc_launch_label(const abc_ctx* c, int j) {
  if (!c || j < 0 || j >= (int)c->launch_labels.size()) return nullptr;
  return c->launch_labels[j].c_str();
}

namespace {

// Adjoint operator set: -dt, and for the face form the kernel of the
// conjugate-transposed section, k'_{l,l'}(p) = conj(k_{l',l}(-p)); first order
// (R = 1) with the aux rescaled by -i conj(a): a -> -conj(a), B -> -B^H.
abc_status build_adjoint(abc_ctx* c) {
  abc_launch& La = c->La;
  La = c->L;
  La.dt = -c->L.dt;
  La.face_fft = nullptr;  // the adjoint kernel is applied directly
  if (c->p.order == ABC_ZEROTH || c->p.order == ABC_FIRST) {
    const int R = c->p.radius, K = 2 * c->p.window + 1;
    const double sgn = c->p.order == ABC_FIRST ? -1.0 : 1.0;
    std::vector<double2> kh(c->face.kernel.size());
    for (int l = 0; l < R; ++l)
      for (int lp = 0; lp < R; ++lp)
        for (int i = 0; i < K; ++i)
          for (int j = 0; j < K; ++j) {
            const abc::cd v = std::conj(c->face.kernel[((lp * R + l) * K + (K - 1 - i)) * K + (K - 1 - j)]);
            kh[((l * R + lp) * K + i) * K + j] = make_double2(sgn * v.real(), sgn * v.imag());
          }
    void* kd = nullptr;
    abc_status st = dev_alloc(c, &kd, kh.size() * sizeof(double2));
    if (st != ABC_OK) return st;
    if (hipMemcpy(kd, kh.data(), kh.size() * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess)
      return fail(ABC_EDEVICE, "hipMemcpy of adjoint kernel failed");
    La.face_ker = static_cast<const double2*>(kd);
    if (c->p.order == ABC_FIRST) La.a_loc[0] = make_double2(-c->L.a_loc[0].x, c->L.a_loc[0].y);
    // the fused kernels' local face value (window 0)
    if (K == 1) La.fused_m0 = La.fused_b0 = kh[0];
  }
  c->adjoint_ready = true;
  return ABC_OK;
}

}  // namespace

abc_status abc_adjoint(abc_ctx* c, const void* psi0, const void* V, int n_steps, int ckpt_stride, int objective,
                       void* grad_psi0, double* grad_V, double* J_out, void* stream) {
  if (!c || !psi0 || !grad_psi0 || !grad_V || !J_out) return fail(ABC_EINVAL, "null argument");
  if (n_steps < 0) return fail(ABC_EINVAL, "n_steps must be >= 0");
  if (objective != ABC_OBJ_PROB && objective != ABC_OBJ_ENERGY) return fail(ABC_EINVAL, "unknown objective");
  const abc_params& p = c->p;
  if (p.dtype != ABC_C128) return fail(ABC_ENOTSUP, "adjoint: complex128 only");
  if (p.batch != 1 || p.meanfield != ABC_MF_NONE) return fail(ABC_ENOTSUP, "adjoint: one orbital, no mean field");
  if (p.order == ABC_SECOND) return fail(ABC_ENOTSUP, "adjoint: not for the second order");
  if ((p.order == ABC_ZEROTH || p.order == ABC_FIRST) && p.form != ABC_FORM_FACES)
    return fail(ABC_ENOTSUP, "adjoint: face form only");
  if (p.order == ABC_FIRST && p.radius != 1) return fail(ABC_ENOTSUP, "adjoint: first order needs R = 1");
  if (!c->adjoint_ready) {
    abc_status st = build_adjoint(c);
    if (st != ABC_OK) return st;
  }
  abc_adjoint_args a{psi0, V, n_steps, ckpt_stride, objective, grad_psi0, grad_V, J_out, c->use_fused};
  std::string err;
  abc_status st = run_adjoint(c->L, c->La, c->S, a, static_cast<hipStream_t>(stream), err);
  if (st != ABC_OK) return fail(st, err);
  return ABC_OK;
}

abc_status abc_effective_potential(abc_ctx* c, const void* psi, const void* V, void* out, void* stream) {
  if (!c || !psi || !out) return fail(ABC_EINVAL, "null argument");
  if (c->p.meanfield != ABC_MF_SKYRME) return fail(ABC_ENOTSUP, "effective potential: ABC_MF_SKYRME contexts only");
  const hipError_t e = skyrme_veff(c->pot, psi, false, c->p.batch, c->p.dtype == ABC_C64, V, out, c->p.t0, c->p.t3,
                                   static_cast<hipStream_t>(stream), nullptr);
  if (e != hipSuccess) return fail(ABC_EDEVICE, std::string("effective potential: ") + hipGetErrorString(e));
  return ABC_OK;
}

namespace {

// checkpoint header: 128 bytes, native (little-endian) layout
struct StateHeader {
  char magic[8];
  int32_t version;
  int32_t nx, ny, nz, radius, order, form, dtype, batch, window, fejer, reserved0;
  double h, dt, s0, s1, s2;
  int64_t step;
  int64_t psi_bytes, aux_bytes;
  char pad[8];
};
static_assert(sizeof(StateHeader) == 128, "checkpoint header size");

StateHeader make_header(const abc_params& p, long long step, int64_t psi_bytes, int64_t aux_bytes) {
  StateHeader hd{};
  std::memcpy(hd.magic, "ABCSTATE", 8);
  hd.version = 1;
  hd.nx = p.nx; hd.ny = p.ny; hd.nz = p.nz; hd.radius = p.radius; hd.order = p.order; hd.form = p.form;
  hd.dtype = p.dtype; hd.batch = p.batch; hd.window = p.window; hd.fejer = p.fejer;
  hd.h = p.h; hd.dt = p.dt; hd.s0 = p.s0; hd.s1 = p.s1; hd.s2 = p.s2;
  hd.step = step;
  hd.psi_bytes = psi_bytes;
  hd.aux_bytes = aux_bytes;
  return hd;
}

int64_t psi_bytes_of(const abc_ctx* c) {
  return (int64_t)c->p.nx * c->p.ny * c->p.nz * c->p.batch * (c->p.dtype == ABC_C64 ? 8 : 16);
}

}  // namespace

abc_status abc_state_save(abc_ctx* c, const void* psi, const void* aux, long long step, const char* path,
                          void* stream) {
  if (!c || !psi || !path) return fail(ABC_EINVAL, "null argument");
  if (c->aux_elems && !aux) return fail(ABC_EINVAL, "this context's state includes the aux buffer");
  const int64_t pb = psi_bytes_of(c), ab = (int64_t)c->aux_elems * 16;
  std::vector<char> buf((size_t)(pb + ab));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(st) != hipSuccess || hipMemcpy(buf.data(), psi, pb, hipMemcpyDeviceToHost) != hipSuccess ||
      (ab && hipMemcpy(buf.data() + pb, aux, ab, hipMemcpyDeviceToHost) != hipSuccess))
    return fail(ABC_EDEVICE, "checkpoint: device copy failed");
  const StateHeader hd = make_header(c->p, step, pb, ab);
  FILE* fp = std::fopen(path, "wb");
  if (!fp) return fail(ABC_EIO, std::string("checkpoint: cannot open ") + path);
  const bool ok = std::fwrite(&hd, sizeof(hd), 1, fp) == 1 && std::fwrite(buf.data(), 1, buf.size(), fp) == buf.size();
  if (std::fclose(fp) != 0 || !ok) return fail(ABC_EIO, std::string("checkpoint: cannot write ") + path);
  return ABC_OK;
}

abc_status abc_state_load(abc_ctx* c, void* psi, void* aux, long long* step, const char* path, void* stream) {
  if (!c || !psi || !path) return fail(ABC_EINVAL, "null argument");
  if (c->aux_elems && !aux) return fail(ABC_EINVAL, "this context's state includes the aux buffer");
  FILE* fp = std::fopen(path, "rb");
  if (!fp) return fail(ABC_EIO, std::string("checkpoint: cannot open ") + path);
  StateHeader hd{};
  if (std::fread(&hd, sizeof(hd), 1, fp) != 1) {
    std::fclose(fp);
    return fail(ABC_EIO, "checkpoint: short header");
  }
  const StateHeader want = make_header(c->p, 0, psi_bytes_of(c), (int64_t)c->aux_elems * 16);
  const char* bad = nullptr;
  if (std::memcmp(hd.magic, want.magic, 8) != 0 || hd.version != want.version) bad = "not a checkpoint of this format";
  else if (hd.nx != want.nx || hd.ny != want.ny || hd.nz != want.nz) bad = "box size";
  else if (hd.radius != want.radius || hd.order != want.order || hd.form != want.form) bad = "radius, order or form";
  else if (hd.dtype != want.dtype || hd.batch != want.batch) bad = "dtype or batch";
  else if (hd.window != want.window || hd.fejer != want.fejer) bad = "face window";
  else if (hd.h != want.h || hd.dt != want.dt) bad = "h or dt";
  else if (hd.s0 != want.s0 || hd.s1 != want.s1 || hd.s2 != want.s2) bad = "interpolation points";
  else if (hd.psi_bytes != want.psi_bytes || hd.aux_bytes != want.aux_bytes) bad = "state sizes";
  if (bad) {
    std::fclose(fp);
    return fail(ABC_EINVAL, std::string("checkpoint does not match the context: ") + bad);
  }
  std::vector<char> buf((size_t)(hd.psi_bytes + hd.aux_bytes));
  const bool ok = std::fread(buf.data(), 1, buf.size(), fp) == buf.size();
  std::fclose(fp);
  if (!ok) return fail(ABC_EIO, "checkpoint: short data");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(st) != hipSuccess ||
      hipMemcpy(psi, buf.data(), hd.psi_bytes, hipMemcpyHostToDevice) != hipSuccess ||
      (hd.aux_bytes && hipMemcpy(aux, buf.data() + hd.psi_bytes, hd.aux_bytes, hipMemcpyHostToDevice) != hipSuccess))
    return fail(ABC_EDEVICE, "checkpoint: device copy failed");
  if (step) *step = hd.step;
  return ABC_OK;
}

namespace {

// the device tallies of the solves: Yukawa, Coulomb iterations, unconverged
abc_status read_tally(const abc_ctx* c, double* t) {
  t[0] = t[1] = t[2] = 0;
  if (!c->pot.tally) return ABC_OK;
  if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(t, c->pot.tally, 3 * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(ABC_EDEVICE, "reading the solves' tallies failed");
  return ABC_OK;
}

}  // namespace

abc_status abc_potential_iterations(const abc_ctx* c, long long* out) {
  if (!c || !out) return fail(ABC_EINVAL, "null argument");
  out[0] = c->pot.solves;
  out[1] = c->pot.iters_y;
  out[2] = c->pot.iters_c;
  if (c->pot.fixed > 0) {
    double t[3];
    const abc_status s = read_tally(c, t);
    if (s != ABC_OK) return s;
    out[1] = (long long)t[0];
    out[2] = (long long)t[1];
  }
  return ABC_OK;
}

abc_status abc_potential_unconverged(const abc_ctx* c, long long* out) {
  if (!c || !out) return fail(ABC_EINVAL, "null argument");
  double t[3];
  const abc_status s = read_tally(c, t);
  if (s != ABC_OK) return s;
  *out = (long long)t[2];
  return ABC_OK;
}

abc_status abc_h2_objective(const abc_params* p, const double* s1, int count, int modes, int nodes, double* out,
                            void* stream) {
  g_last_error.clear();
  if (!p || !s1 || !out) return fail(ABC_EINVAL, "null argument");
  if (count < 1 || modes < 4 || modes > 4096 || nodes < 16 || nodes > (1 << 24))
    return fail(ABC_EINVAL, "H2 objective: count >= 1, 4 <= modes <= 4096, 16 <= nodes <= 2^24");
  abc_status st = check_params(*p);
  if (st != ABC_OK) return st;
  if (p->order != ABC_FIRST || p->form != ABC_FORM_FACES || p->radius != 1)
    return fail(ABC_ENOTSUP, "H2 objective: first-order face form with R = 1 only");
  for (int c = 0; c < count; ++c)
    if (!(s1[c] > 0) || !std::isfinite(s1[c])) return fail(ABC_EINVAL, "H2 objective: points must be positive");
  std::string err;
  st = run_h2_objective(*p, s1, count, modes, nodes, out, static_cast<hipStream_t>(stream), err);
  if (st != ABC_OK) return fail(st, err);
  return ABC_OK;
}

abc_status abc_diagnostics(abc_ctx* c, const void* psi, const void* aux, const void* V, double* out, void* stream) {
  if (!c || !psi || !out) return fail(ABC_EINVAL, "null argument");
  hipError_t e = launch_diagnostics(c->L, c->S, psi, static_cast<const double2*>(aux), V, out,
                                    static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(ABC_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return ABC_OK;
}

}  // extern "C"

namespace {

// Reduction partials of abc_diagnostics_noalloc: a fixed device array, one
// copy per GPU, held until the process ends.  Host code never uses its name
// as an address (that would be the host-side stand-in); the device address
// is looked up once per device and kept.
constexpr int kNoallocMaxBatch = 64;
constexpr size_t kNoallocScratchDoubles = (size_t)kNoallocMaxBatch * (256 + 64) * 4;
__device__ __align__(256) double scratch[kNoallocScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// device address of this device's copy of the array (first call on a
// device: hipGetSymbolAddress with that device current)
abc_status noalloc_scratch(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(ABC_EDEVICE, "abc_diagnostics_noalloc: no current device (or device index >= 64)");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(ABC_EDEVICE, std::string("abc_diagnostics_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return ABC_OK;
}

}  // namespace

extern "C" {

abc_status abc_diagnostics_noalloc(abc_ctx* c, const void* psi, const void* aux, const void* V, double* out,
                                   void* stream) {
  if (!c || !psi || !out) return fail(ABC_EINVAL, "null argument");
  if (diag_partial_doubles(c->p.batch) > kNoallocScratchDoubles)
    return fail(ABC_EINVAL, "abc_diagnostics_noalloc: batch " + std::to_string(c->p.batch) +
                                " exceeds the fixed scratch, which holds the partials of at most " +
                                std::to_string(kNoallocMaxBatch) + " orbitals");
  double* red = nullptr;
  abc_status s = noalloc_scratch(&red);
  if (s != ABC_OK) return s;
  // every partial the finishing pass reads is written by this call's own
  // reduction blocks first, so nothing needs clearing between calls
  hipError_t e = launch_diagnostics(c->L, c->S, psi, static_cast<const double2*>(aux), V, out,
                                    static_cast<hipStream_t>(stream), red);
  if (e != hipSuccess) return fail(ABC_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return ABC_OK;
}

abc_status abc_export(const abc_ctx* c, int which, void* host_out, size_t n) {
  if (!c || !host_out) return fail(ABC_EINVAL, "null argument");
  if (which == 0) {
    if (c->face.kernel.size() > n) return fail(ABC_EINVAL, "buffer too small");
    std::memcpy(host_out, c->face.kernel.data(), c->face.kernel.size() * sizeof(abc::cd));
    return ABC_OK;
  }
  if (which == 1) {
    if (!c->box_mat) return fail(ABC_EINVAL, "no box-form matrix");
    const size_t cnt = abc::box_mat_elems(c->p.order, c->n_gamma);
    if (cnt > n) return fail(ABC_EINVAL, "buffer too small");
    if (hipMemcpy(host_out, c->box_mat, cnt * 16, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(ABC_EDEVICE, "hipMemcpy failed");
    return ABC_OK;
  }
  if (which == 3) {
    if (!c->box_mat) return fail(ABC_EINVAL, "no box-form matrix");
    if (n < 2) return fail(ABC_EINVAL, "buffer too small");
    abc::cd* o = static_cast<abc::cd*>(host_out);
    o[0] = abc::cd((double)c->n_gamma, (double)c->box_rank);
    o[1] = abc::cd(c->box_bound, 0.0);
    return ABC_OK;
  }
  if (which == 2) {
    const int R = c->p.radius;
    if ((size_t)2 * R * R > n) return fail(ABC_EINVAL, "buffer too small");
    abc::cd* o = static_cast<abc::cd*>(host_out);
    for (int i = 0; i < R * R; ++i) { o[i] = c->face.a[i]; o[R * R + i] = c->face.q[i]; }
    return ABC_OK;
  }
  return fail(ABC_EINVAL, "unknown export");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Tile-depth tuner and batches of uneven boxes
// ---------------------------------------------------------------------------

namespace {

// mean milliseconds per step of `run(n)` over a few steps, after a warm-up
template <typename F>
abc_status time_steps(F run, hipStream_t st, float* ms_out) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(ABC_EDEVICE, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return fail(ABC_EDEVICE, "hipEventCreate failed");
  }
  hipError_t e = run(2);
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  if (e == hipSuccess) e = run(6);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (e != hipSuccess) return fail(ABC_EDEVICE, std::string("tuner timing: ") + hipGetErrorString(e));
  *ms_out = ms / 6;
  return ABC_OK;
}

// saved copies of states advanced by the tuner, restored afterwards
struct Saved {
  std::vector<std::pair<void*, void*>> items;  // (user, copy)
  std::vector<size_t> bytes;
  ~Saved() {
    for (auto& it : items) (void)hipFree(it.second);
  }
  abc_status save(void* p, size_t n, hipStream_t st) {
    if (!p || !n) return ABC_OK;
    void* c = nullptr;
    if (hipMalloc(&c, n) != hipSuccess) return fail(ABC_ENOMEM, "tuner: hipMalloc of a state copy failed");
    items.push_back({p, c});
    bytes.push_back(n);
    if (hipMemcpyAsync(c, p, n, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return fail(ABC_EDEVICE, "tuner: state copy failed");
    return ABC_OK;
  }
  abc_status restore(hipStream_t st) {
    for (size_t i = 0; i < items.size(); ++i)
      if (hipMemcpyAsync(items[i].first, items[i].second, bytes[i], hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(ABC_EDEVICE, "tuner: state restore failed");
    if (hipStreamSynchronize(st) != hipSuccess) return fail(ABC_EDEVICE, "tuner: synchronise failed");
    return ABC_OK;
  }
};

size_t psi_bytes(const abc_ctx* c) {
  return (size_t)c->L.g.npts * c->p.batch * (c->p.dtype == ABC_C64 ? 8 : 16);
}

}  // namespace

abc_status abc_tune(abc_ctx* c, void* psi, void* aux, const void* V, void* stream, int* tz_out) {
  if (!c || !psi) return fail(ABC_EINVAL, "null argument");
  if (c->aux_elems && !aux) return fail(ABC_EINVAL, "first and second order need the aux buffer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!c->use_fused || c->orb || c->L.fused_stages != 2) {
    if (tz_out) *tz_out = c->use_fused ? c->L.fused_tz : 0;
    return ABC_OK;
  }
  Saved sv;
  abc_status s = sv.save(psi, psi_bytes(c), st);
  if (s == ABC_OK) s = sv.save(aux, c->aux_elems * sizeof(double2), st);
  if (s != ABC_OK) return s;
  int best = c->L.fused_tz;
  float best_ms = 1e30f;
  for (int tz : {4, 8, 16}) {
    if (!fused_tz_valid(c->L, tz)) continue;
    c->L.fused_tz = tz;
    float ms = 0;
    s = time_steps([&](int n) { return launch_step_fused(c->L, c->S, psi, static_cast<double2*>(aux), V, n, st); },
                   st, &ms);
    if (s != ABC_OK) return s;
    if (ms < best_ms) {
      best_ms = ms;
      best = tz;
    }
  }
  c->L.fused_tz = best;
  if (tz_out) *tz_out = best;
  return sv.restore(st);
}

struct abc_batch {
  std::vector<abc_ctx*> inst;
  struct Group {
    int order = 0, dtype = 0, tz = 8;
    std::vector<int> idx;
    void* host = nullptr;  // pinned descriptor staging
    void* dev = nullptr;   // descriptors of eager calls
    void* gdev = nullptr;  // descriptors baked into the cached graph
    hipEvent_t copied = nullptr;
    bool pending = false;
  };
  std::vector<Group> groups;
  std::vector<int> fallback;  // instances stepped through abc_step one by one
  // groups after the first run on a second stream (default priority),
  // forked from and joined back to the caller's stream, so that the groups'
  // launches overlap and fill each other's last rounds of workgroups
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> key;
  int key_n = -1;
  hipStream_t key_stream = nullptr;
};

void abc_destroy_batch(abc_batch* b) {
  if (!b) return;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->fork) hipEventDestroy(b->fork);
  if (b->join) hipEventDestroy(b->join);
  if (b->side) hipStreamDestroy(b->side);
  for (auto& g : b->groups) {
    if (g.copied) hipEventDestroy(g.copied);
    if (g.host) hipHostFree(g.host);
    if (g.dev) hipFree(g.dev);
    if (g.gdev) hipFree(g.gdev);
  }
  for (abc_ctx* c : b->inst) abc_destroy(c);
  delete b;
}

abc_status abc_setup_batch(const abc_params* ps, int n, abc_batch** out) {
  g_last_error.clear();
  if (!ps || !out || n < 1) return fail(ABC_EINVAL, "null argument or empty batch");
  *out = nullptr;
  abc_batch* b = new abc_batch();
  for (int i = 0; i < n; ++i) {
    abc_ctx* c = nullptr;
    if (ps[i].meanfield == ABC_MF_SKYRME) {
      abc_destroy_batch(b);
      return fail(ABC_ENOTSUP, "instance " + std::to_string(i) + ": the Skyrme mean field is not batched");
    }
    // the batch launch runs the two-stage kernels: an instance on the
    // automatic path takes them when they cover it
    abc_params pi = ps[i];
    if (pi.path == ABC_PATH_AUTO && fused_supported(pi, nullptr)) pi.path = ABC_PATH_FUSED;
    abc_status st = abc_setup(&pi, &c);
    if (st != ABC_OK) {
      const std::string msg = "instance " + std::to_string(i) + ": " + g_last_error;
      abc_destroy_batch(b);
      return fail(st, msg);
    }
    b->inst.push_back(c);
    if (!(c->use_fused && !c->orb && c->L.fused_stages == 2)) {
      b->fallback.push_back(i);
      continue;
    }
    abc_batch::Group* g = nullptr;
    for (auto& gg : b->groups)
      if (gg.order == c->p.order && gg.dtype == c->p.dtype) g = &gg;
    if (!g) {
      b->groups.emplace_back();
      g = &b->groups.back();
      g->order = c->p.order;
      g->dtype = c->p.dtype;
    }
    g->idx.push_back(i);
  }
  if (b->groups.size() > 1 &&
      (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
       hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
       hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess)) {
    abc_destroy_batch(b);
    return fail(ABC_EDEVICE, "batch stream or events");
  }
  for (auto& g : b->groups) {
    for (int i : g.idx) g.tz = std::min(g.tz, fused_max_tz(g.order, b->inst[i]->p.nz));
    for (int i : g.idx) b->inst[i]->L.fused_tz = g.tz;
    const size_t bytes = fused_batch_desc_bytes((int)g.idx.size());
    if (hipHostMalloc(&g.host, bytes) != hipSuccess || hipMalloc(&g.dev, bytes) != hipSuccess ||
        hipMalloc(&g.gdev, bytes) != hipSuccess || hipEventCreate(&g.copied) != hipSuccess) {
      abc_destroy_batch(b);
      return fail(ABC_ENOMEM, "batch descriptor buffers");
    }
  }
  *out = b;
  return ABC_OK;
}

size_t abc_batch_aux_elems(const abc_batch* b, int i) {
  if (!b || i < 0 || i >= (int)b->inst.size()) return 0;
  return b->inst[i]->aux_elems;
}

int abc_batch_launch_groups(const abc_batch* b) { return b ? (int)b->groups.size() : 0; }

int abc_batch_tile_depth(const abc_batch* b, int group) {
  if (!b || group < 0 || group >= (int)b->groups.size()) return 0;
  return b->groups[group].tz;
}

namespace {

std::vector<FusedMember> members(abc_batch* b, const abc_batch::Group& g, void* const* psi, void* const* aux,
                                 const void* const* V) {
  std::vector<FusedMember> m;
  for (int i : g.idx)
    m.push_back({&b->inst[i]->L, &b->inst[i]->S, psi[i], aux ? static_cast<double2*>(aux[i]) : nullptr,
                 V ? V[i] : nullptr});
  return m;
}

abc_status check_batch_args(abc_batch* b, void* const* psi, void* const* aux) {
  if (!b || !psi) return fail(ABC_EINVAL, "null argument");
  for (size_t i = 0; i < b->inst.size(); ++i) {
    if (!psi[i]) return fail(ABC_EINVAL, "null psi for instance " + std::to_string(i));
    if (b->inst[i]->aux_elems && (!aux || !aux[i]))
      return fail(ABC_EINVAL, "instance " + std::to_string(i) + " needs its aux buffer");
  }
  return ABC_OK;
}

// enqueue every launch of an n-step batch call; descriptors are already in
// `use_graph ? gdev : dev`
abc_status enqueue_batch(abc_batch* b, void* const* psi, void* const* aux, const void* const* V, int n,
                         hipStream_t st, bool use_graph, const std::vector<int>& totals) {
  const bool two = b->side && b->groups.size() > 1;
  if (two && (hipEventRecord(b->fork, st) != hipSuccess || hipStreamWaitEvent(b->side, b->fork, 0) != hipSuccess))
    return fail(ABC_EDEVICE, "batch stream fork failed");
  for (size_t k = 0; k < b->groups.size(); ++k) {
    auto& g = b->groups[k];
    hipError_t e = launch_batch_fused(members(b, g, psi, aux, V), g.tz, use_graph ? g.gdev : g.dev, totals[k], n,
                                      two && k > 0 ? b->side : st, nullptr);
    if (e != hipSuccess) return fail(ABC_EDEVICE, std::string("batch launch: ") + hipGetErrorString(e));
  }
  if (two && (hipEventRecord(b->join, b->side) != hipSuccess || hipStreamWaitEvent(st, b->join, 0) != hipSuccess))
    return fail(ABC_EDEVICE, "batch stream join failed");
  for (int i : b->fallback) {
    abc_status s = abc_step(b->inst[i], psi[i], aux ? aux[i] : nullptr, V ? V[i] : nullptr, n, st);
    if (s != ABC_OK) return s;
  }
  return ABC_OK;
}

}  // namespace

abc_status abc_step_batch(abc_batch* b, void* const* psi, void* const* aux, const void* const* V, int n_steps,
                          int flags, void* stream) {
  abc_status s = check_batch_args(b, psi, aux);
  if (s != ABC_OK) return s;
  if (n_steps < 0) return fail(ABC_EINVAL, "n_steps must be >= 0");
  if (n_steps == 0) return ABC_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool graph = (flags & ABC_BATCH_GRAPH) != 0;
  if (graph && !st) return fail(ABC_EINVAL, "graph capture needs a non-default stream");
  std::vector<int> totals(b->groups.size());
  if (!graph) {
    for (size_t k = 0; k < b->groups.size(); ++k) {
      auto& g = b->groups[k];
      // the staging buffer is reused once its previous copy has completed
      if (g.pending && hipEventSynchronize(g.copied) != hipSuccess) return fail(ABC_EDEVICE, "event wait failed");
      totals[k] = fused_batch_build(members(b, g, psi, aux, V), g.host, n_steps);
      if (hipMemcpyAsync(g.dev, g.host, fused_batch_desc_bytes((int)g.idx.size()), hipMemcpyHostToDevice, st) !=
              hipSuccess ||
          hipEventRecord(g.copied, st) != hipSuccess)
        return fail(ABC_EDEVICE, "descriptor upload failed");
      g.pending = true;
    }
    return enqueue_batch(b, psi, aux, V, n_steps, st, false, totals);
  }
  // graph mode: one captured graph per (buffers, n_steps, stream), replayed
  std::vector<const void*> key;
  for (size_t i = 0; i < b->inst.size(); ++i) {
    key.push_back(psi[i]);
    key.push_back(aux ? aux[i] : nullptr);
    key.push_back(V ? V[i] : nullptr);
  }
  if (!(b->exec && key == b->key && n_steps == b->key_n && st == b->key_stream)) {
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    for (size_t k = 0; k < b->groups.size(); ++k) {
      auto& g = b->groups[k];
      if (g.pending && hipEventSynchronize(g.copied) != hipSuccess) return fail(ABC_EDEVICE, "event wait failed");
      g.pending = false;
      totals[k] = fused_batch_build(members(b, g, psi, aux, V), g.host, n_steps);
      if (hipMemcpy(g.gdev, g.host, fused_batch_desc_bytes((int)g.idx.size()), hipMemcpyHostToDevice) != hipSuccess)
        return fail(ABC_EDEVICE, "descriptor upload failed");
    }
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return fail(ABC_EDEVICE, "hipStreamBeginCapture failed");
    s = enqueue_batch(b, psi, aux, V, n_steps, st, true, totals);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (s != ABC_OK) {
      if (graph) hipGraphDestroy(graph);
      return s;
    }
    if (e != hipSuccess || !graph) return fail(ABC_EDEVICE, "hipStreamEndCapture failed");
    if (hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      hipGraphDestroy(graph);
      return fail(ABC_EDEVICE, "hipGraphInstantiate failed");
    }
    b->graph = graph;
    b->key = key;
    b->key_n = n_steps;
    b->key_stream = st;
  }
  if (hipGraphLaunch(b->exec, st) != hipSuccess) return fail(ABC_EDEVICE, "hipGraphLaunch failed");
  return ABC_OK;
}

abc_status abc_tune_batch(abc_batch* b, void* const* psi, void* const* aux, const void* const* V, void* stream) {
  abc_status s = check_batch_args(b, psi, aux);
  if (s != ABC_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Saved sv;
  for (size_t i = 0; i < b->inst.size(); ++i) {
    s = sv.save(psi[i], psi_bytes(b->inst[i]), st);
    if (s == ABC_OK && aux) s = sv.save(aux[i], b->inst[i]->aux_elems * sizeof(double2), st);
    if (s != ABC_OK) return s;
  }
  // On every exit, each instance's tile depth is its group's (the depth the
  // group's kernels are instantiated at) and the callers' states are back.
  auto finish = [&](abc_status r) {
    for (auto& g : b->groups)
      for (int i : g.idx) b->inst[i]->L.fused_tz = g.tz;
    const abc_status rr = sv.restore(st);
    return r != ABC_OK ? r : rr;
  };
  for (auto& g : b->groups) {
    int max_tz = 16;
    for (int i : g.idx) max_tz = std::min(max_tz, fused_max_tz(g.order, b->inst[i]->p.nz));
    const auto m = members(b, g, psi, aux, V);
    int best = g.tz;
    float best_ms = 1e30f;
    for (int tz : {4, 8, 16}) {
      if (tz > max_tz) continue;
      for (int i : g.idx) b->inst[i]->L.fused_tz = tz;
      float ms = 0;
      s = time_steps(
          [&](int n) {
            if (g.pending && hipEventSynchronize(g.copied) != hipSuccess) return hipErrorUnknown;
            const int total = fused_batch_build(m, g.host, n);
            hipError_t e = hipMemcpyAsync(g.dev, g.host, fused_batch_desc_bytes((int)g.idx.size()),
                                          hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipEventRecord(g.copied, st);
            g.pending = true;
            if (e == hipSuccess) e = launch_batch_fused(m, tz, g.dev, total, n, st, nullptr);
            return e;
          },
          st, &ms);
      if (s != ABC_OK) return finish(s);
      if (ms < best_ms) {
        best_ms = ms;
        best = tz;
      }
    }
    g.tz = best;
  }
  // a cached graph was captured with the old depths
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  return finish(ABC_OK);
}
