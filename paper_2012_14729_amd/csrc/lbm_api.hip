// C-ABI host code of the phase-field LBM library: argument validation,
// derived constants, workspace layout, launch sequencing, checkpoints and
// kernel timing.  Declarations and semantics: include/lbm.h.
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "../../include/lbm.h"
#include "lbm_internal.hpp"

using namespace pflbm;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

}  // namespace

int pflbm::set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

namespace {

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(LBM_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool finite(double v) { return std::isfinite(v); }

int validate(const lbm_params* p) {
  if (!p) return fail(LBM_E_INVAL, "params is NULL");
  if (p->nx < 8 || p->ny < 8) return fail(LBM_E_INVAL, "nx, ny must be >= 8 (got %d, %d)", p->nx, p->ny);
  if ((((long long)p->nx + 63) / 64 * 64) * p->ny >= (1LL << 31))
    return fail(LBM_E_INVAL, "grid too large (the padded plane must hold fewer than 2^31 nodes)");
  if (p->wall_x < 0 || p->wall_x > 2 || p->wall_y < 0 || p->wall_y > 2)
    return fail(LBM_E_INVAL, "wall_x, wall_y must be 0 (periodic), 1 (no-slip) or 2 (free-slip)");
  if (p->wall_x && p->wall_y && (p->u_wall_lo != 0.0 || p->u_wall_hi != 0.0))
    return fail(LBM_E_INVAL, "moving walls need exactly one walled axis");
  if ((p->wall_x == 2 || p->wall_y == 2) && (p->u_wall_lo != 0.0 || p->u_wall_hi != 0.0))
    return fail(LBM_E_INVAL, "free-slip walls do not move");
  const double v[] = {p->u_wall_lo, p->u_wall_hi, p->rho1, p->rho2, p->nu1, p->nu2, p->sigma,
                      p->W,         p->M,         p->tau_h, p->gx,  p->gy,  p->eps_n};
  for (double d : v)
    if (!finite(d)) return fail(LBM_E_INVAL, "non-finite parameter");
  if (!(p->rho1 > 0 && p->rho2 > 0)) return fail(LBM_E_INVAL, "densities must be positive");
  if (!(p->nu1 > 0 && p->nu2 > 0)) return fail(LBM_E_INVAL, "viscosities must be positive (tau_f > 1/2)");
  if (!(p->sigma >= 0)) return fail(LBM_E_INVAL, "sigma must be >= 0");
  if (!(p->W > 0)) return fail(LBM_E_INVAL, "W must be > 0");
  if (!(p->M >= 0)) return fail(LBM_E_INVAL, "M must be >= 0");
  if (!(p->tau_h > 0.5)) return fail(LBM_E_INVAL, "tau_h must be > 1/2");
  if (!(p->eps_n > 0)) return fail(LBM_E_INVAL, "eps_n must be > 0");
  if (!std::isnan(p->rho0) && !finite(p->rho0)) return fail(LBM_E_INVAL, "rho0 must be finite or NaN");
  return LBM_OK;
}

}  // namespace

// Derived coefficients (Sec. II.A Eq. 6; Sec. III after Eqs. 36 and 40).
Phys pflbm::derive_phys(const lbm_params* p, double rho0) {
  Phys c{};
  const double beta = 3.0 * p->sigma / (4.0 * p->W);
  const double kappa = 3.0 * p->W * p->sigma / 8.0;
  const double tau2 = p->tau_h * p->tau_h - p->tau_h + 1.0 / 6.0, tau1 = p->tau_h - 0.5;
  const double mu1 = p->rho1 * p->nu1, mu2 = p->rho2 * p->nu2;
  c.rho_a = (float)(0.5 * (p->rho1 + p->rho2));
  c.rho_b = (float)(0.5 * (p->rho1 - p->rho2));
  c.mu_a = (float)(0.5 * (mu1 + mu2));
  c.mu_b = (float)(0.5 * (mu1 - mu2));
  c.beta4 = (float)(4.0 * beta);
  c.kappa = (float)kappa;
  c.sigma_half = (float)(0.5 * p->sigma);
  c.eps2 = (float)(p->eps_n * p->eps_n);
  c.eta = (float)(p->M / ((1.0 / 3.0) * tau1));
  c.a_h = (float)(3.0 * tau2 / (p->tau_h * tau1));
  c.inv_tau_h = (float)(1.0 / p->tau_h);
  c.gx = (float)p->gx;
  c.gy = (float)p->gy;
  c.rho0 = (float)rho0;
  c.uw_lo = (float)p->u_wall_lo;
  c.uw_hi = (float)p->u_wall_hi;
  c.wall_x = p->wall_x != 0;   // walled axis (no-slip or free-slip; the kind is in Grid)
  c.wall_y = p->wall_y != 0;
  c.beta4_d = 4.0 * beta;
  c.kappa_d = kappa;
  c.sigma_half_d = 0.5 * p->sigma;
  c.eps2_d = p->eps_n * p->eps_n;
  c.rho2_d = p->rho2;
  c.drho_half_d = 0.5 * (p->rho1 - p->rho2);
  c.mu2_d = mu2;
  c.dmu_half_d = 0.5 * (mu1 - mu2);
  c.eta_d = p->M / ((1.0 / 3.0) * tau1);
  c.a_h_d = 3.0 * tau2 / (p->tau_h * tau1);
  c.inv_tau_h_d = 1.0 / p->tau_h;
  c.gx_d = p->gx;
  c.gy_d = p->gy;
  c.rho0_d = rho0;
  c.uw_lo_d = p->u_wall_lo;
  c.uw_hi_d = p->u_wall_hi;
  return c;
}

namespace {

Phys derive(const lbm_params* p, double rho0) { return derive_phys(p, rho0); }

struct Layout {
  Grid g;
  size_t off_s[2], off_phi, off_status, off_partial, off_sum, total;
};

constexpr int kPartials = 512;

Layout layout_for(const lbm_params* p) {
  Layout L{};
  L.g.nx = p->nx;
  L.g.ny = p->ny;
  L.g.pitch = (int)align_up((size_t)p->nx, 64);
  L.g.ncx = L.g.pitch / 64;
  L.g.ps = (long long)L.g.pitch * p->ny;
  L.g.rowe = L.g.ncx * kSegE;
  L.g.fast = fast_bits(L.g.ps);
  if (const char* e = std::getenv("PFLBM_GENERAL_PATH")) {   // diagnostics: 1 every tile general, 2 no wrapped path
    if (e[0] == '1') L.g.fast = 0;
    if (e[0] == '2') L.g.fast &= kFastInterior;
  }
  L.g.slip_x = p->wall_x == 2;
  L.g.slip_y = p->wall_y == 2;
  const size_t sbytes = (size_t)kNPL * (size_t)L.g.ps * sizeof(float);
  size_t o = 0;
  for (int b = 0; b < 2; ++b) { L.off_s[b] = o; o = align_up(o + sbytes, kAlign); }
  L.off_phi = o; o = align_up(o + (size_t)L.g.ps * sizeof(double), kAlign);
  L.off_status = o; o = align_up(o + 64 * sizeof(int), kAlign);
  L.off_partial = o; o = align_up(o + kPartials * sizeof(double), kAlign);
  L.off_sum = o; o = align_up(o + sizeof(double), kAlign);
  L.total = o;
  return L;
}

}  // namespace

struct lbm_sim {
  lbm_params p;
  Layout L;
  Phys c;
  char* ws;
  int cur;          // population buffer holding the current state
  int shape;        // tile shape of the step kernels (index into kShapeTX/kShapeTY)
  int64_t step;
  int timing;
  int64_t timing_base;   // step count when timing was last set: the first step after it is timed
  // ring of event quadruples, one per timed step: the fused kernel's start
  // and stop, the order-parameter kernel's start and stop, each taken from
  // the kernel's dispatch; a slot is drained (its elapsed times added) before
  // reuse or on query
  static constexpr int kRing = 512;
  hipEvent_t ev[kRing][4];
  int ev_pending[kRing];
  int ev_next;
  double t_ms[2];
  int64_t t_n[2];
  float* S(int b) const { return (float*)(ws + L.off_s[b]); }
  double* phi() const { return (double*)(ws + L.off_phi); }
  size_t state_floats() const { return (size_t)kNPL * (size_t)L.g.ps; }
  int* status() const { return (int*)(ws + L.off_status); }
};

namespace {

StepArgs step_args(const lbm_sim* s) {
  StepArgs a{};
  a.sin = s->S(s->cur);
  a.sout = s->S(1 - s->cur);
  a.phi = s->phi();
  a.status = s->status();
  a.g = s->L.g;
  a.c = s->c;
  return a;
}

// Add the elapsed times of ring slot `j` (both kernels) if it holds a step.
int drain_slot(lbm_sim* s, int j) {
  if (!s->ev_pending[j]) return LBM_OK;
  HIPCHK(hipEventSynchronize(s->ev[j][3]));
  for (int k = 0; k < 2; ++k) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, s->ev[j][2 * k], s->ev[j][2 * k + 1]));
    s->t_ms[k] += ms;
    s->t_n[k] += 1;
  }
  s->ev_pending[j] = 0;
  return LBM_OK;
}

int drain_all(lbm_sim* s) {
  for (int j = 0; j < lbm_sim::kRing; ++j)
    if (int r = drain_slot(s, j)) return r;
  return LBM_OK;
}

// The next ring slot for a timed step (drained first).
int timer_slot(lbm_sim* s, int* slot) {
  const int j = s->ev_next;
  s->ev_next = (j + 1) % lbm_sim::kRing;
  if (int r = drain_slot(s, j)) return r;
  *slot = j;
  return LBM_OK;
}

}  // namespace

int pflbm::sim_params(const lbm_sim* s, lbm_params* out) {
  if (!s || !out) return fail(LBM_E_INVAL, "NULL argument");
  *out = s->p;
  return LBM_OK;
}

Phys pflbm::sim_phys(const lbm_sim* s) { return s->c; }

int pflbm::sim_view(const lbm_sim* s, SimView* v) {
  if (!s || !v) return fail(LBM_E_INVAL, "NULL argument");
  v->s = s->S(s->cur);
  v->phi = s->phi();
  v->g = s->L.g;
  return LBM_OK;
}

extern "C" {

const char* lbm_last_error(void) { return g_err; }
const char* lbm_version(void) { return "pflbm-mi355x 0.1 (gfx950)"; }

int lbm_workspace_bytes(const lbm_params* p, size_t* bytes) {
  if (int r = validate(p)) return r;
  if (!bytes) return fail(LBM_E_INVAL, "bytes is NULL");
  *bytes = layout_for(p).total;
  return LBM_OK;
}

int lbm_init(lbm_sim** out, const lbm_params* p, void* d_ws, size_t ws_bytes, const float* d_phi0,
             const float* d_ux0, const float* d_uy0, void* stream) {
  if (!out) return fail(LBM_E_INVAL, "sim is NULL");
  *out = nullptr;
  if (int r = validate(p)) return r;
  if (!d_ws || ((uintptr_t)d_ws % kAlign) != 0) return fail(LBM_E_INVAL, "workspace must be non-NULL and 256-byte aligned");
  if (!d_phi0) return fail(LBM_E_INVAL, "phi0 is NULL");
  if ((d_ux0 == nullptr) != (d_uy0 == nullptr)) return fail(LBM_E_INVAL, "give both u0 components or neither");
  Layout L = layout_for(p);
  if (ws_bytes < L.total) return fail(LBM_E_INVAL, "workspace too small: %zu < %zu", ws_bytes, L.total);
  lbm_sim* s = new (std::nothrow) lbm_sim();
  if (!s) return fail(LBM_E_INVAL, "out of host memory");
  s->p = *p;
  s->L = L;
  s->ws = (char*)d_ws;
  s->cur = 0;
  s->step = 0;
  s->shape = 0;
  if (const char* e = std::getenv("PFLBM_TILE")) {   // diagnostics: tile shape of a periodic lattice's step
    const int sh = atoi(e);
    if (sh < 0 || sh >= kNumShapes) {
      delete s;
      return fail(LBM_E_INVAL, "PFLBM_TILE must be 0..%d", kNumShapes - 1);
    }
    if (!p->wall_x && !p->wall_y) s->shape = sh;
  }
  hipStream_t st = (hipStream_t)stream;
  Phys c = derive(p, 0.0);
  // node-local initial populations go to state array 1, the stored layout to array 0
  hipError_t e = launch_init(d_phi0, d_ux0, d_uy0, s->S(1), s->S(0), s->phi(), L.g, c, st);
  if (e == hipSuccess) e = launch_fill_int(s->status(), 0, 64, st);
  double rho0 = p->rho0;
  if (e == hipSuccess && std::isnan(p->rho0)) {
    // A12: rho0 = mean of rho(phi0), fixed for the run
    double* partial = (double*)(s->ws + L.off_partial);
    double* sum = (double*)(s->ws + L.off_sum);
    e = launch_phi_sum(s->phi(), L.g, partial, kPartials, sum, st);
    double hsum = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hsum, sum, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    const double mean_phi = hsum / ((double)p->nx * p->ny);
    rho0 = p->rho1 * (1.0 + mean_phi) / 2.0 + p->rho2 * (1.0 - mean_phi) / 2.0;
  }
  if (e != hipSuccess) {
    delete s;
    return fail(LBM_E_HIP, "lbm_init: %s", hipGetErrorString(e));
  }
  s->c = derive(p, rho0);
  *out = s;
  return LBM_OK;
}

int lbm_step(lbm_sim* s, int32_t nsteps, int32_t form, void* stream) {
  if (!s) return fail(LBM_E_INVAL, "sim is NULL");
  if (nsteps < 0) return fail(LBM_E_INVAL, "nsteps must be >= 0");
  if (form < 0 || form >= LBM_NUM_FORMS) return fail(LBM_E_INVAL, "bad force form %d", form);
  hipStream_t st = (hipStream_t)stream;
  for (int32_t n = 0; n < nsteps; ++n) {
    StepArgs a = step_args(s);
    const bool timed = s->timing && (s->step - s->timing_base) % s->timing == 0;
    int slot = -1;
    if (timed)
      if (int r = timer_slot(s, &slot)) return r;
    hipEvent_t* ev = slot >= 0 ? s->ev[slot] : nullptr;
    HIPCHK(launch_fused(form, s->shape, a, st, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr));
    HIPCHK(launch_phi(a.sout, s->phi(), s->phi(), s->L.g, s->c.wall_x, s->c.wall_y, s->shape, st,
                      ev ? ev[2] : nullptr, ev ? ev[3] : nullptr));
    if (slot >= 0) s->ev_pending[slot] = 1;
    s->cur = 1 - s->cur;
    s->step += 1;
  }
  return LBM_OK;
}

int lbm_moments(lbm_sim* s, int32_t form, float* d_phi, float* d_rho, float* d_ux, float* d_uy, float* d_p,
                void* stream) {
  if (!s) return fail(LBM_E_INVAL, "sim is NULL");
  if (form < 0 || form >= LBM_NUM_FORMS) return fail(LBM_E_INVAL, "bad force form %d", form);
  MomentArgs m{d_phi, d_rho, d_ux, d_uy, d_p, nullptr};
  HIPCHK(launch_moments(form, step_args(s), m, (hipStream_t)stream));
  return LBM_OK;
}

int lbm_hydro_pressure(lbm_sim* s, int32_t form, float* d_ph, void* stream) {
  if (!s || !d_ph) return fail(LBM_E_INVAL, "NULL argument");
  if (form < 0 || form >= LBM_NUM_FORMS) return fail(LBM_E_INVAL, "bad force form %d", form);
  MomentArgs m{nullptr, nullptr, nullptr, nullptr, nullptr, d_ph};
  HIPCHK(launch_moments(form, step_args(s), m, (hipStream_t)stream));
  return LBM_OK;
}

int lbm_status(lbm_sim* s, int32_t* diverged, void* stream) {
  if (!s || !diverged) return fail(LBM_E_INVAL, "NULL argument");
  int h = 0;
  HIPCHK(hipMemcpyAsync(&h, s->status(), sizeof(int), hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  *diverged = h ? 1 : 0;
  return h ? fail(LBM_E_DIVERGED, "simulation produced non-finite values") : LBM_OK;
}

int lbm_get_step(const lbm_sim* s, int64_t* step) {
  if (!s || !step) return fail(LBM_E_INVAL, "NULL argument");
  *step = s->step;
  return LBM_OK;
}

// blob: [state array, 21 interleaved planes][phi FP64 plane][status][zeros]
int lbm_state_bytes(const lbm_sim* s, size_t* bytes) {
  if (!s || !bytes) return fail(LBM_E_INVAL, "NULL argument");
  *bytes = s->state_floats() * sizeof(float) + (size_t)s->L.g.ps * sizeof(double) + kAlign;
  return LBM_OK;
}

int lbm_save(lbm_sim* s, void* d_blob, void* stream) {
  if (!s || !d_blob) return fail(LBM_E_INVAL, "NULL argument");
  const size_t sb = s->state_floats() * sizeof(float), pb = (size_t)s->L.g.ps * sizeof(double);
  char* b = (char*)d_blob;
  const void* src[3] = {s->S(s->cur), s->phi(), s->status()};
  void* dst[3] = {b, b + sb, b + sb + pb};
  const size_t bytes[3] = {sb, pb, sizeof(int)};
  // the rest of the blob is zero, so equal states give equal blobs
  HIPCHK(launch_copies(src, dst, bytes, 3, b + sb + pb + sizeof(int), kAlign - sizeof(int), (hipStream_t)stream));
  return LBM_OK;
}

int lbm_restore(lbm_sim* s, const void* d_blob, void* stream) {
  if (!s || !d_blob) return fail(LBM_E_INVAL, "NULL argument");
  const size_t sb = s->state_floats() * sizeof(float), pb = (size_t)s->L.g.ps * sizeof(double);
  const char* b = (const char*)d_blob;
  const void* src[3] = {b, b + sb, b + sb + pb};
  void* dst[3] = {s->S(s->cur), s->phi(), s->status()};
  const size_t bytes[3] = {sb, pb, sizeof(int)};
  HIPCHK(launch_copies(src, dst, bytes, 3, nullptr, 0, (hipStream_t)stream));
  return LBM_OK;
}

int lbm_step_blobs(lbm_sim* s, const void* d_blob_in, void* d_blob_out, int32_t form, void* stream) {
  if (!s || !d_blob_in || !d_blob_out) return fail(LBM_E_INVAL, "NULL argument");
  if (form < 0 || form >= LBM_NUM_FORMS) return fail(LBM_E_INVAL, "bad force form %d", form);
  const size_t sb = s->state_floats() * sizeof(float), pb = (size_t)s->L.g.ps * sizeof(double);
  const size_t tot = sb + pb + kAlign;
  const char* bi = (const char*)d_blob_in;
  char* bo = (char*)d_blob_out;
  if (bi < bo + tot && bo < bi + tot) return fail(LBM_E_INVAL, "the two blobs must not overlap");
  hipStream_t st = (hipStream_t)stream;
  // the divergence flag carries over (the kernels then add to it), the tail is zero
  const void* src[1] = {bi + sb + pb};
  void* dst[1] = {bo + sb + pb};
  const size_t bytes[1] = {sizeof(int)};
  HIPCHK(launch_copies(src, dst, bytes, 1, bo + sb + pb + sizeof(int), kAlign - sizeof(int), st));
  StepArgs a = step_args(s);
  a.sin = (const float*)bi;
  a.sout = (float*)bo;
  a.phi = (const double*)(bi + sb);
  a.status = (int*)(bo + sb + pb);
  HIPCHK(launch_fused(form, s->shape, a, st));
  HIPCHK(launch_phi(a.sout, (const double*)(bi + sb), (double*)(bo + sb), s->L.g, s->c.wall_x, s->c.wall_y, s->shape,
                    st));
  return LBM_OK;
}

int lbm_set_timing(lbm_sim* s, int32_t enable) {
  if (!s) return fail(LBM_E_INVAL, "sim is NULL");
  if (enable < 0) return fail(LBM_E_INVAL, "timing period must be >= 0");
  if (enable && !s->ev[0][0]) {   // create the event ring on first use
    for (int j = 0; j < lbm_sim::kRing; ++j)
      for (int e = 0; e < 4; ++e) HIPCHK(hipEventCreate(&s->ev[j][e]));
  }
  if (s->ev[0][0])
    if (int r = drain_all(s)) return r;
  s->timing = enable;   // 0: off; k: every k-th step, starting with the next one
  s->timing_base = s->step;
  s->t_ms[0] = s->t_ms[1] = 0.0;
  s->t_n[0] = s->t_n[1] = 0;
  return LBM_OK;
}

int lbm_kernel_time(lbm_sim* s, int32_t kernel, double* total_ms, int64_t* launches) {
  if (!s || !total_ms || !launches || kernel < 0 || kernel > 1) return fail(LBM_E_INVAL, "bad argument");
  if (s->ev[0][0])
    if (int r = drain_all(s)) return r;
  *total_ms = s->t_ms[kernel];
  *launches = s->t_n[kernel];
  return LBM_OK;
}

int lbm_destroy(lbm_sim* s) {
  if (!s) return LBM_OK;
  for (int j = 0; j < lbm_sim::kRing; ++j)
    for (int e = 0; e < 4; ++e)
      if (s->ev[j][e]) (void)hipEventDestroy(s->ev[j][e]);
  delete s;
  return LBM_OK;
}

}  // extern "C"
