// Hand-written adjoint of one time step of the phase-field LBM
// (arXiv:2012.14729, Sec. II-IV), and of the initial state.
//
// The adjoint acts on the physical pre-collision state of a step: f_i, h_i
// (i = 0..8) and J = (phi u) of the previous step, nine + nine + two FP64
// values per node.  Given lambda_{n+1} = dL/ds_{n+1} it returns
// lambda_n = (ds_{n+1}/ds_n)^T lambda_{n+1} and accumulates dL/dsigma and
// dL/dM per node.
//
// Layout: every field is a dense row-major FP64 array.  Fields that the step
// evaluates beyond the domain live on explicitly extended grids: "e1" holds
// one ghost layer ((nx+2) x (ny+2)), "e2" two ((nx+4) x (ny+4)).  Ghost values
// come from the extension rules of Sec. IV (periodic wrap; even reflection
// of phi and u_ghost = 2 u_w - u(mirror) at a half-way wall), so every
// stencil and every transposed stencil is a plain gather on these grids.  The
// boundary logic lives only in the extension maps and in their transposes
// (fold-back sums over the ghost preimages of each node).
//
// Forward recomputation: k_adj_unpack, k_adj_fa .. k_adj_fe.
// Backward:              k_adj_b1 .. k_adj_b7.
// All arithmetic is FP64.
#include <cmath>
#include <new>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.hpp"

using namespace pflbm;

namespace {

constexpr int kB = 256;
constexpr double CS2 = 1.0 / 3.0;

struct AGrid {
  int nx, ny, wx, wy;
  Grid sg;          // layout of the simulation's state arrays
};

__device__ __forceinline__ int i0(const AGrid& g, int x, int y) { return y * g.nx + x; }
__device__ __forceinline__ int i1(const AGrid& g, int x, int y) { return (y + 1) * (g.nx + 2) + (x + 1); }
__device__ __forceinline__ int i2(const AGrid& g, int x, int y) { return (y + 2) * (g.nx + 4) + (x + 2); }

// extension map along one axis: position p in [-k, n+k) -> node, with a sign
// flip count for the velocity ghost rule
__device__ __forceinline__ int ext_map(int p, int n, int wall, int& refl) {
  refl = 0;
  if (p >= 0 && p < n) return p;
  if (!wall) return p < 0 ? p + n : p - n;
  refl = 1;
  return p < 0 ? -1 - p : 2 * n - 1 - p;
}

// preimages of node c in [-k, n+k) under ext_map; returns count (<= 3)
__device__ __forceinline__ int preimages(int c, int n, int wall, int k, int* p, int* refl) {
  int m = 0;
  p[m] = c; refl[m] = 0; ++m;
  if (!wall) {
    if (c - n >= -k) { p[m] = c - n; refl[m] = 0; ++m; }
    if (c + n < n + k) { p[m] = c + n; refl[m] = 0; ++m; }
  } else {
    if (-1 - c >= -k) { p[m] = -1 - c; refl[m] = 1; ++m; }
    if (2 * n - 1 - c < n + k) { p[m] = 2 * n - 1 - c; refl[m] = 1; ++m; }
  }
  return m;
}

struct ABuf {
  // physical state (input of the adjoint step), interior
  double *f, *h, *J;                       // 9, 9, 2 planes
  // forward intermediates
  double *phi, *phie2;                     // interior, e2
  double *G1, *L1, *mu1, *T1, *n1, *s1;    // e1 (G1, n1: 2 planes; T1: 3 planes)
  double *Fsf, *F, *rho, *muv, *tauf, *u, *gr, *P, *Q, *ue1, *Q1, *D, *dQ, *divn;   // interior (ue1, Q1: e1)
  // adjoint intermediates
  double *lf, *lh;                         // 9 planes each, interior (partial lambda of the pre-collision state)
  double *lP, *lrho, *lu, *lF, *lgr, *lphi, *lD, *lQ;   // interior
  double *lue1, *lphie1;                   // e1
  double *lG1, *lL1;                       // e1 (lG1 2 planes)
  double *lmun;                            // interior: adjoint of mu at the node from h^eq
  double *lphie2;                          // e2
  double *gsig, *gM;                       // per-node gradient densities (e1-sized, accumulated over steps)
};

struct ACon {
  double beta4, kappa, sigma, eps2, eta, detadM, a_h, inv_tau_h;
  double rho2, drho_h, mu2, dmu_h, gx, gy, rho0, uw_lo, uw_hi;
  int form;
};

// ---------------------------------------------------------------------------
// Forward recomputation
// ---------------------------------------------------------------------------

// Physical pre-collision state from the stored single-lattice state (pull
// form of streaming, Eq. 43 pre-applied): f_i = ft_i + w_i P at the source,
// h_i pulled for i >= 1, h_0 = phi - sum_{i>=1} h_i, J.
__global__ __launch_bounds__(kB) void k_adj_unpack(const float* __restrict__ S, const double* __restrict__ phis, AGrid g, ABuf b) {
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= g.nx * g.ny) return;
  const int x = k % g.nx, y = k / g.nx;
  const int N = g.nx * g.ny;
  // every pull is loaded before any result is stored, so the loads are in
  // flight together (the source of a pull is one node away: one wrap)
  float fv[9], pv[9], hv[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    int sx = x - cx(i), sy = y - cy(i), slot = i;
    bool bounce = false;
    if (sx < 0 || sx >= g.nx) { if (g.wx) bounce = true; else sx = sx < 0 ? sx + g.nx : sx - g.nx; }
    if (sy < 0 || sy >= g.ny) { if (g.wy) bounce = true; else sy = sy < 0 ? sy + g.ny : sy - g.ny; }
    const unsigned nb = bounce ? nbase(g.sg, x, y) : nbase(g.sg, sx, sy);
    if (bounce) slot = opp(i);
    fv[i] = S[nb + (unsigned)((kPF + slot) * 64)];
    pv[i] = S[nb + (unsigned)(kPP * 64)];
    hv[i] = i > 0 ? S[nb + (unsigned)((kPH + slot) * 64)] : 0.0f;
  }
  double hsum = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    b.f[(size_t)i * N + k] = (double)fv[i] + wtd(i) * (double)pv[i];
    if (i > 0) {
      const double h = (double)hv[i];
      b.h[(size_t)i * N + k] = h;
      hsum += h;
    }
  }
  const unsigned on = nbase(g.sg, x, y);
  b.h[k] = phis[(long long)y * g.sg.pitch + x] - hsum;
  b.J[k] = (double)S[on + (unsigned)(kPJ * 64)];
  b.J[N + k] = (double)S[on + (unsigned)((kPJ + 1) * 64)];
}

__global__ __launch_bounds__(kB) void k_adj_fa(AGrid g, ABuf b) {   // phi = sum_i h_i (Eq. 37), then the e2 extension
  const int ne = (g.nx + 4) * (g.ny + 4);
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= ne) return;
  const int ex = k % (g.nx + 4) - 2, ey = k / (g.nx + 4) - 2;
  int r;
  const int x = ext_map(ex, g.nx, g.wx, r), y = ext_map(ey, g.ny, g.wy, r);
  const int N = g.nx * g.ny, n = i0(g, x, y);
  double s = 0.0;
  for (int i = 0; i < 9; ++i) s += b.h[(size_t)i * N + n];
  b.phie2[k] = s;
  if (ex == x && ey == y) b.phi[n] = s;
}

// On e1: grad, lap (Eqs. 41-42), mu_phi (Eq. 2) and the form's node fields.
__global__ __launch_bounds__(kB) void k_adj_fb(AGrid g, ACon c, ABuf b) {
  const int ne = (g.nx + 2) * (g.ny + 2);
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= ne) return;
  const int x = k % (g.nx + 2) - 1, y = k / (g.nx + 2) - 1;
  const double pc = b.phie2[i2(g, x, y)];
  double gx = 0, gy = 0, l = 0;
  for (int i = 1; i < 9; ++i) {
    const double v = b.phie2[i2(g, x + cx(i), y + cy(i))];
    gx += wtd(i) * cx(i) * v;
    gy += wtd(i) * cy(i) * v;
    l += wtd(i) * (v - pc);
  }
  gx *= 3.0; gy *= 3.0; l *= 6.0;
  b.G1[k] = gx;
  b.G1[ne + k] = gy;
  b.L1[k] = l;
  b.mu1[k] = c.beta4 * pc * (pc * pc - 1.0) - c.kappa * l;
  if (c.form == 0) {        // STF-1: T = -kappa G (x) G  (F = div T)
    b.T1[k] = -c.kappa * gx * gx; b.T1[ne + k] = -c.kappa * gx * gy; b.T1[2 * ne + k] = -c.kappa * gy * gy;
  } else if (c.form == 1) { // STF-2: T = kappa (|G|^2 I - G (x) G)
    b.T1[k] = c.kappa * gy * gy; b.T1[ne + k] = -c.kappa * gx * gy; b.T1[2 * ne + k] = c.kappa * gx * gx;
  } else if (c.form >= 6) { // CSF: n = G / s, s = sqrt(|G|^2 + eps^2)
    const double s = sqrt(gx * gx + gy * gy + c.eps2);
    b.s1[k] = s;
    b.n1[k] = gx / s;
    b.n1[ne + k] = gy / s;
  }
}

// Interior: F_sf (Sec. II.B), F_g (Eq. 8), rho, mu, tau_f (A6), u and P (Eq. 37), Q = phi u.
__global__ __launch_bounds__(kB) void k_adj_fc(AGrid g, ACon c, ABuf b) {
  const int N = g.nx * g.ny;
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  const int x = k % g.nx, y = k / g.nx;
  const int ne = (g.nx + 2) * (g.ny + 2);
  const int e = i1(g, x, y);
  const double phi = b.phi[k], gx = b.G1[e], gy = b.G1[ne + e], l = b.L1[e], mu = b.mu1[e];
  // the populations are read before anything is stored (stores and loads
  // share one in-order counter, and the compiler cannot move a load above a
  // store to a buffer it cannot prove disjoint)
  double fv[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) fv[i] = b.f[(size_t)i * N + k];
  double fx = 0, fy = 0, dn = 0;
  if (c.form <= 1) {
    for (int i = 1; i < 9; ++i) {
      const int q = i1(g, x + cx(i), y + cy(i));
      fx += wtd(i) * (cx(i) * b.T1[q] + cy(i) * b.T1[ne + q]);
      fy += wtd(i) * (cx(i) * b.T1[ne + q] + cy(i) * b.T1[2 * ne + q]);
    }
    fx *= 3.0; fy *= 3.0;
  } else if (c.form == 2 || c.form == 5) {   // -phi grad mu  |  kappa phi grad lap
    const double* fld = c.form == 2 ? b.mu1 : b.L1;
    double ax = 0, ay = 0;
    for (int i = 1; i < 9; ++i) {
      const double v = fld[i1(g, x + cx(i), y + cy(i))];
      ax += wtd(i) * cx(i) * v;
      ay += wtd(i) * cy(i) * v;
    }
    ax *= 3.0; ay *= 3.0;
    const double k2 = c.form == 2 ? -phi : c.kappa * phi;
    fx = k2 * ax; fy = k2 * ay;
  } else if (c.form == 3) {
    fx = mu * gx; fy = mu * gy;
  } else if (c.form == 4) {
    fx = -c.kappa * gx * l; fy = -c.kappa * gy * l;
  } else {
    for (int i = 1; i < 9; ++i) {
      const int q = i1(g, x + cx(i), y + cy(i));
      dn += wtd(i) * (cx(i) * b.n1[q] + cy(i) * b.n1[ne + q]);
    }
    dn *= 3.0;
    b.divn[k] = dn;
    if (c.form == 6) {
      const double g2 = gx * gx + gy * gy;
      fx = -c.kappa * g2 * b.n1[e] * dn; fy = -c.kappa * g2 * b.n1[ne + e] * dn;
    } else {
      fx = -0.5 * c.sigma * gx * dn; fy = -0.5 * c.sigma * gy * dn;
    }
  }
  b.Fsf[k] = fx; b.Fsf[N + k] = fy;
  const double rho = c.rho2 + c.drho_h * (1.0 + phi);
  const double muv = c.mu2 + c.dmu_h * (1.0 + phi);
  const double Fx = fx + (rho - c.rho0) * c.gx, Fy = fy + (rho - c.rho0) * c.gy;
  b.F[k] = Fx; b.F[N + k] = Fy;
  b.rho[k] = rho; b.muv[k] = muv; b.tauf[k] = 0.5 + muv / (CS2 * rho);
  double jx = 0, jy = 0, S = 0;
  for (int i = 0; i < 9; ++i) {
    const double fi = fv[i];
    jx += cx(i) * fi; jy += cy(i) * fi; S += fi;
  }
  const double ux = (jx + 0.5 * CS2 * Fx) / (CS2 * rho), uy = (jy + 0.5 * CS2 * Fy) / (CS2 * rho);
  b.u[k] = ux; b.u[N + k] = uy;
  const double grx = c.drho_h * gx, gry = c.drho_h * gy;
  b.gr[k] = grx; b.gr[N + k] = gry;
  b.P[k] = S + 0.5 * CS2 * (ux * grx + uy * gry);
  b.Q[k] = phi * ux; b.Q[N + k] = phi * uy;
}

// e1: ghost velocity (A9) and the node field phi u for div(phi u).
__global__ __launch_bounds__(kB) void k_adj_fd(AGrid g, ACon c, ABuf b) {
  const int ne = (g.nx + 2) * (g.ny + 2), N = g.nx * g.ny;
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= ne) return;
  const int ex = k % (g.nx + 2) - 1, ey = k / (g.nx + 2) - 1;
  int rx, ry;
  const int x = ext_map(ex, g.nx, g.wx, rx), y = ext_map(ey, g.ny, g.wy, ry);
  double ux = b.u[i0(g, x, y)], uy = b.u[N + i0(g, x, y)];
  // x-extension first, then y (the ghost velocity of a wall is 2 u_w - u)
  if (rx) { const double w = ex < 0 ? c.uw_lo : c.uw_hi; ux = -ux; uy = 2.0 * w - uy; }
  if (ry) { const double w = ey < 0 ? c.uw_lo : c.uw_hi; ux = 2.0 * w - ux; uy = -uy; }
  b.ue1[k] = ux; b.ue1[ne + k] = uy;
  const double ph = b.phie2[i2(g, ex, ey)];
  b.Q1[k] = ph * ux; b.Q1[ne + k] = ph * uy;
}

__global__ __launch_bounds__(kB) void k_adj_fe(AGrid g, ABuf b) {   // D = div(phi u) (Eq. 41), dQ = Q - J (A4)
  const int N = g.nx * g.ny, ne = (g.nx + 2) * (g.ny + 2);
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  const int x = k % g.nx, y = k / g.nx;
  double d = 0;
  for (int i = 1; i < 9; ++i) {
    const int q = i1(g, x + cx(i), y + cy(i));
    d += wtd(i) * (cx(i) * b.Q1[q] + cy(i) * b.Q1[ne + q]);
  }
  b.D[k] = 3.0 * d;
  b.dQ[k] = b.Q[k] - b.J[k];
  b.dQ[N + k] = b.Q[N + k] - b.J[N + k];
}

// ---------------------------------------------------------------------------
// Backward
// ---------------------------------------------------------------------------

// Streaming and both collisions transposed (Eqs. 29-36, 43), node-local.
// lam: lambda_{n+1} (9 f, 9 h, 2 J planes).  Writes the partial adjoints of
// the pre-collision populations and of every node quantity they depend on.
// lam and lam_out may be the same array (in-place step): not restrict-qualified.
__global__ __launch_bounds__(kB) void k_adj_b1(AGrid g, ACon c, ABuf b, const double* lam, double* lam_out) {
  const int N = g.nx * g.ny;
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  const int x = k % g.nx, y = k / g.nx;
  const double phi = b.phi[k], rho = b.rho[k], tauf = b.tauf[k], ux = b.u[k], uy = b.u[N + k];
  const double Fx = b.F[k], Fy = b.F[N + k], grx = b.gr[k], gry = b.gr[N + k], P = b.P[k];
  const double mu = b.mu1[i1(g, x, y)];
  const double om = 1.0 / tauf, cf = 1.0 - 0.5 * om, omh = c.inv_tau_h, cfh = 1.0 - 0.5 * omh;
  const double usq = ux * ux + uy * uy;
  const double dqx = b.dQ[k], dqy = b.dQ[N + k], D = b.D[k];
  double lP = 0, lrho = 0, lux = 0, luy = 0, lFx = 0, lFy = 0, lgx = 0, lgy = 0, lphi = 0, lmu = 0, lD = 0;
  double ldqx = 0, ldqy = 0, lom = 0, gM = 0;
  // transpose of streaming: the post-collision value of direction i at x
  // became population i at x + c_i, or population opp(i) at x at a wall.
  // All adjoint values and populations are loaded before the per-direction
  // stores below (separate buffers), so the loads are in flight together.
  bool hit_[9];
  double cuw_[9], lfp_[9], lhp_[9], fi_[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    int tx = x + cx(i), ty = y + cy(i);
    bool hit = false;
    double cuw = 0;
    if (tx < 0 || tx >= g.nx) { if (g.wx) { hit = true; cuw = cy(i) * (tx < 0 ? c.uw_lo : c.uw_hi); } else tx = tx < 0 ? tx + g.nx : tx - g.nx; }
    if (ty < 0 || ty >= g.ny) { if (g.wy) { hit = true; cuw = cx(i) * (ty < 0 ? c.uw_lo : c.uw_hi); } else ty = ty < 0 ? ty + g.ny : ty - g.ny; }
    const int slot = hit ? opp(i) : i;
    const int tgt = hit ? k : i0(g, tx, ty);
    hit_[i] = hit;
    cuw_[i] = cuw;
    lfp_[i] = lam[(size_t)slot * N + tgt];
    lhp_[i] = lam[(size_t)(9 + slot) * N + tgt];
    fi_[i] = b.f[(size_t)i * N + k];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const bool hit = hit_[i];
    const double cuw = cuw_[i], lfp = lfp_[i], lhp = lhp_[i];
    if (hit) {   // f_opp = f_i^+ - 2 w_i rho c_i.u_w ; h_opp = h_i^+ - 6 w_i phi c_i.u_w
      lrho += -2.0 * wtd(i) * cuw * lfp;
      lphi += -6.0 * wtd(i) * cuw * lhp;
    }
    // flow collision f^+ = (1 - om) f + om feq + cf F_i
    const double fi = fi_[i];
    const double cu = cx(i) * ux + cy(i) * uy;
    const double si = 3.0 * cu + 4.5 * cu * cu - 1.5 * usq;
    const double feq = wtd(i) * (P + CS2 * rho * si);
    const double Vx = wtd(i) * (1.0 + si) * Fx + wtd(i) * si * CS2 * grx;
    const double Vy = wtd(i) * (1.0 + si) * Fy + wtd(i) * si * CS2 * gry;
    const double Fi = (cx(i) - ux) * Vx + (cy(i) - uy) * Vy;
    b.lf[(size_t)i * N + k] = (1.0 - om) * lfp;
    lom += lfp * (feq - fi - 0.5 * Fi);
    const double lfeq = om * lfp, lFi = cf * lfp;
    lP += wtd(i) * lfeq;
    lrho += wtd(i) * CS2 * si * lfeq;
    double lsi = wtd(i) * CS2 * rho * lfeq;
    lux += -Vx * lFi;
    luy += -Vy * lFi;
    const double lVx = (cx(i) - ux) * lFi, lVy = (cy(i) - uy) * lFi;
    lFx += wtd(i) * (1.0 + si) * lVx;
    lFy += wtd(i) * (1.0 + si) * lVy;
    lgx += wtd(i) * si * CS2 * lVx;
    lgy += wtd(i) * si * CS2 * lVy;
    lsi += wtd(i) * (Fx * lVx + Fy * lVy) + wtd(i) * CS2 * (grx * lVx + gry * lVy);
    lux += lsi * (3.0 * cx(i) + 9.0 * cu * cx(i) - 3.0 * ux);
    luy += lsi * (3.0 * cy(i) + 9.0 * cu * cy(i) - 3.0 * uy);
    // order-parameter collision h^+ = (1 - omh) h + omh heq + cfh H_i
    b.lh[(size_t)i * N + k] = (1.0 - omh) * lhp;
    const double lheq = omh * lhp, lH = cfh * lhp;
    const double wb = i == 0 ? wtd(0) - 1.0 : wtd(i);
    if (i == 0) lphi += lheq;
    else {
      lphi += 3.0 * wtd(i) * cu * lheq;
      lux += 3.0 * wtd(i) * phi * cx(i) * lheq;
      luy += 3.0 * wtd(i) * phi * cy(i) * lheq;
    }
    lmu += c.eta * wb * lheq;
    gM += mu * wb * lheq * c.detadM;
    lD += wb * c.a_h * lH;
    ldqx += 3.0 * wtd(i) * cx(i) * lH;
    ldqy += 3.0 * wtd(i) * cy(i) * lH;
  }
  (void)D; (void)dqx; (void)dqy;
  // tau_f = 1/2 + mu/(cs^2 rho), om = 1/tau_f
  const double ltau = -lom / (tauf * tauf);
  lrho += -b.muv[k] / (CS2 * rho * rho) * ltau;
  lphi += c.dmu_h * ltau / (CS2 * rho);
  // P = S + cs^2/2 u.grad rho  (S = sum f)
  lux += 0.5 * CS2 * grx * lP;
  luy += 0.5 * CS2 * gry * lP;
  lgx += 0.5 * CS2 * ux * lP;
  lgy += 0.5 * CS2 * uy * lP;
  // J_{n+1} = Q, dQ = Q - J_n, Q = phi u
  const double lQx = lam[(size_t)18 * N + k] + ldqx, lQy = lam[(size_t)19 * N + k] + ldqy;
  lam_out[(size_t)18 * N + k] = -ldqx;
  lam_out[(size_t)19 * N + k] = -ldqy;
  lux += phi * lQx;
  luy += phi * lQy;
  lphi += ux * lQx + uy * lQy;
  b.lP[k] = lP; b.lrho[k] = lrho; b.lu[k] = lux; b.lu[N + k] = luy;
  b.lF[k] = lFx; b.lF[N + k] = lFy; b.lgr[k] = lgx; b.lgr[N + k] = lgy;
  b.lphi[k] = lphi; b.lD[k] = lD; b.lQ[k] = lQx; b.lQ[N + k] = lQy;
  b.lmun[k] = lmu;
  b.gM[i1(g, x, y)] += gM;
}

// e1: transpose of D = div(Q1) and of Q1 = phi_e1 u_e1.
__global__ __launch_bounds__(kB) void k_adj_b2(AGrid g, ABuf b) {
  const int ne = (g.nx + 2) * (g.ny + 2);
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= ne) return;
  const int ex = k % (g.nx + 2) - 1, ey = k / (g.nx + 2) - 1;
  double lqx = 0, lqy = 0;
  for (int i = 1; i < 9; ++i) {   // D(x) = 3 sum_i w_i c_i . Q1(x + c_i)
    // out-of-range neighbours load node 0 and contribute zero (all loads in flight together)
    const int x = ex - cx(i), y = ey - cy(i);
    const bool ok = x >= 0 && x < g.nx && y >= 0 && y < g.ny;
    const double v = b.lD[ok ? i0(g, x, y) : 0];
    const double ld = 3.0 * wtd(i) * (ok ? v : 0.0);
    lqx += cx(i) * ld;
    lqy += cy(i) * ld;
  }
  const double ph = b.phie2[i2(g, ex, ey)];
  b.lue1[k] = ph * lqx;
  b.lue1[ne + k] = ph * lqy;
  b.lphie1[k] = b.ue1[k] * lqx + b.ue1[ne + k] * lqy;
}

// Interior: fold the ghost-velocity adjoints back (A9), then transpose
// u = (j + cs^2 F/2)/(cs^2 rho), P's S = sum f, F = F_sf + (rho - rho0) g, rho(phi).
__global__ __launch_bounds__(kB) void k_adj_b3(AGrid g, ACon c, ABuf b) {
  const int N = g.nx * g.ny, ne = (g.nx + 2) * (g.ny + 2);
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  const int x = k % g.nx, y = k / g.nx;
  const int e = i1(g, x, y);
  // Every value this thread reads is loaded before its first store: stores
  // and loads share one in-order counter, and the compiler cannot move a
  // load above a store to a buffer it cannot prove disjoint.
  double lux = b.lu[k], luy = b.lu[N + k];
  int px[3], rx[3], py[3], ry[3];
  const int mx = preimages(x, g.nx, g.wx, 1, px, rx), my = preimages(y, g.ny, g.wy, 1, py, ry);
  for (int a = 0; a < mx; ++a)
    for (int bb = 0; bb < my; ++bb) {
      const int q = i1(g, px[a], py[bb]);
      const double sg = ((rx[a] + ry[bb]) & 1) ? -1.0 : 1.0;
      lux += sg * b.lue1[q];
      luy += sg * b.lue1[ne + q];
    }
  const double rho = b.rho[k], ux = b.u[k], uy = b.u[N + k];
  const double lF0x = b.lF[k], lF0y = b.lF[N + k], lrho0 = b.lrho[k], lS = b.lP[k], lphi0 = b.lphi[k];
  double lfv[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) lfv[i] = b.lf[(size_t)i * N + k];
  const bool cpf1_pf2 = c.form == 2 || c.form == 5;
  double fv[9];
  if (cpf1_pf2) {
    const double* fld = c.form == 2 ? b.mu1 : b.L1;
#pragma unroll
    for (int i = 1; i < 9; ++i) fv[i] = fld[i1(g, x + cx(i), y + cy(i))];
  }
  const bool sig_f = !(c.form == 2 || c.form == 3);
  const double fsx = sig_f ? b.Fsf[k] : 0.0, fsy = sig_f ? b.Fsf[N + k] : 0.0;
  const double gsig0 = sig_f ? b.gsig[e] : 0.0;
  const double lgr0x = b.lgr[k], lgr0y = b.lgr[N + k];
  double g1x = 0.0, g1y = 0.0, n1x = 0.0, n1y = 0.0;
  if (c.form >= 6) {
    g1x = b.G1[e]; g1y = b.G1[ne + e];
    if (c.form == 6) { n1x = b.n1[e]; n1y = b.n1[ne + e]; }
  }

  const double ljx = lux / (CS2 * rho), ljy = luy / (CS2 * rho);
  double lFx = lF0x + 0.5 * lux / rho, lFy = lF0y + 0.5 * luy / rho;
  double lrho = lrho0 - (ux * lux + uy * luy) / rho;
#pragma unroll
  for (int i = 0; i < 9; ++i) b.lf[(size_t)i * N + k] = lfv[i] + (cx(i) * ljx + cy(i) * ljy + lS);
  lrho += c.gx * lFx + c.gy * lFy;
  b.lF[k] = lFx; b.lF[N + k] = lFy;   // now the adjoint of F_sf
  double lphi = lphi0 + c.drho_h * lrho;
  // point-wise parts of the force transposes that touch phi (CPF-1, PF-2)
  if (cpf1_pf2) {
    double ax = 0, ay = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      ax += wtd(i) * cx(i) * fv[i];
      ay += wtd(i) * cy(i) * fv[i];
    }
    const double s = c.form == 2 ? -3.0 : 3.0 * c.kappa;
    lphi += s * (ax * lFx + ay * lFy);
  }
  b.lphi[k] = lphi;
  // sigma enters F_sf linearly for every form except through mu (CPF forms)
  if (sig_f) b.gsig[e] = gsig0 + (fsx * lFx + fsy * lFy) / c.sigma;
  // grad rho = (rho1 - rho2)/2 G  -> lambda_G contribution kept in lgr
  b.lgr[k] = lgr0x * c.drho_h;
  b.lgr[N + k] = lgr0y * c.drho_h;
  if (c.form >= 6) {   // adjoint of div n at the node (stored in lD, free after b2)
    b.lD[k] = c.form == 6 ? -c.kappa * (g1x * g1x + g1y * g1y) * (n1x * lFx + n1y * lFy)
                          : -0.5 * c.sigma * (g1x * lFx + g1y * lFy);
  }
}

// e1: adjoints of the e1 node fields G1, L1, mu1 from the force (per form),
// from grad rho and from h^eq.
__global__ __launch_bounds__(kB) void k_adj_b4(AGrid g, ACon c, ABuf b) {
  const int ne = (g.nx + 2) * (g.ny + 2), N = g.nx * g.ny;
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= ne) return;
  const int ex = k % (g.nx + 2) - 1, ey = k / (g.nx + 2) - 1;
  const bool in = ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny;
  const int n = in ? i0(g, ex, ey) : 0;
  const double gx = b.G1[k], gy = b.G1[ne + k], l = b.L1[k], mu = b.mu1[k];
  double lgx = 0, lgy = 0, ll = 0, lmu = 0;
  if (in) {
    lgx += b.lgr[n];
    lgy += b.lgr[N + n];
    lmu += b.lmun[n];
  }
  const double lFx = in ? b.lF[n] : 0.0, lFy = in ? b.lF[N + n] : 0.0;
  if (c.form <= 1) {
    // F(x) = 3 sum_i w_i [c_ix T(x + c_i) ; ...]: transpose gathers from x = e - c_i
    double ltxx = 0, ltxy = 0, ltyy = 0;
    for (int i = 1; i < 9; ++i) {
      // out-of-range neighbours load node 0 and contribute zero, so all
      // loads are issued together instead of one branch at a time
      const int x = ex - cx(i), y = ey - cy(i);
      const bool ok = x >= 0 && x < g.nx && y >= 0 && y < g.ny;
      const int m = ok ? i0(g, x, y) : 0;
      const double w = 3.0 * wtd(i);
      const double lx = b.lF[m], ly = b.lF[N + m];
      const double ax = ok ? lx : 0.0, ay = ok ? ly : 0.0;
      ltxx += w * cx(i) * ax;
      ltxy += w * (cy(i) * ax + cx(i) * ay);
      ltyy += w * cy(i) * ay;
    }
    if (c.form == 0) {
      lgx += -c.kappa * (2.0 * gx * ltxx + gy * ltxy);
      lgy += -c.kappa * (gx * ltxy + 2.0 * gy * ltyy);
    } else {
      lgx += c.kappa * (-gy * ltxy + 2.0 * gx * ltyy);
      lgy += c.kappa * (2.0 * gy * ltxx - gx * ltxy);
    }
  } else if (c.form == 2 || c.form == 5) {
    // CPF-1: F = -phi grad mu1 ; PF-2: F = kappa phi grad L1
    double acc = 0;
    for (int i = 1; i < 9; ++i) {
      const int x = ex - cx(i), y = ey - cy(i);
      const bool ok = x >= 0 && x < g.nx && y >= 0 && y < g.ny;
      const int m = ok ? i0(g, x, y) : 0;
      const double lx = b.lF[m], ly = b.lF[N + m], pm = b.phi[m];
      acc += 3.0 * wtd(i) * (cx(i) * (ok ? lx : 0.0) + cy(i) * (ok ? ly : 0.0)) * pm;
    }
    if (c.form == 2) lmu += -acc;
    else ll += c.kappa * acc;
  } else if (c.form == 3) {   // CPF-2: F = mu G
    lmu += gx * lFx + gy * lFy;
    lgx += mu * lFx;
    lgy += mu * lFy;
  } else if (c.form == 4) {   // PF-1: F = -kappa G L
    lgx += -c.kappa * l * lFx;
    lgy += -c.kappa * l * lFy;
    ll += -c.kappa * (gx * lFx + gy * lFy);
  } else {                    // CSF: div n gathers, then n(G)
    double lnx = 0, lny = 0;
    for (int i = 1; i < 9; ++i) {
      const int x = ex - cx(i), y = ey - cy(i);
      const bool ok = x >= 0 && x < g.nx && y >= 0 && y < g.ny;
      const double v = b.lD[ok ? i0(g, x, y) : 0];
      const double ld = 3.0 * wtd(i) * (ok ? v : 0.0);
      lnx += cx(i) * ld;
      lny += cy(i) * ld;
    }
    if (in) {
      const double dn = b.divn[n];
      if (c.form == 6) {
        const double g2 = gx * gx + gy * gy, nx = b.n1[k], ny = b.n1[ne + k];
        lnx += -c.kappa * g2 * dn * lFx;
        lny += -c.kappa * g2 * dn * lFy;
        const double t = -c.kappa * 2.0 * dn * (nx * lFx + ny * lFy);
        lgx += t * gx;
        lgy += t * gy;
      } else {
        lgx += -0.5 * c.sigma * dn * lFx;
        lgy += -0.5 * c.sigma * dn * lFy;
      }
    }
    const double s = b.s1[k], gn = (gx * lnx + gy * lny) / (s * s * s);
    lgx += lnx / s - gx * gn;
    lgy += lny / s - gy * gn;
  }
  // mu1 = 4 beta phi (phi^2 - 1) - kappa L1
  ll += -c.kappa * lmu;
  const double ph = b.phie2[i2(g, ex, ey)];
  b.lphie1[k] += c.beta4 * (3.0 * ph * ph - 1.0) * lmu;
  b.gsig[k] += lmu * mu / c.sigma;
  b.lG1[k] = lgx;
  b.lG1[ne + k] = lgy;
  b.lL1[k] = ll;
}

// e2: transposes of G1 = grad(phie2), L1 = lap(phie2), plus the e1 phi adjoints.
__global__ __launch_bounds__(kB) void k_adj_b6(AGrid g, ABuf b) {
  const int n2 = (g.nx + 4) * (g.ny + 4), ne = (g.nx + 2) * (g.ny + 2);
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= n2) return;
  const int zx = k % (g.nx + 4) - 2, zy = k / (g.nx + 4) - 2;
  const bool in1 = zx >= -1 && zx <= g.nx && zy >= -1 && zy <= g.ny;
  double acc = 0;
  for (int i = 1; i < 9; ++i) {   // out-of-range: load position 0, contribute zero
    const int ex = zx - cx(i), ey = zy - cy(i);
    const bool ok = ex >= -1 && ex <= g.nx && ey >= -1 && ey <= g.ny;
    const int e = ok ? i1(g, ex, ey) : 0;
    const double gx = b.lG1[e], gy = b.lG1[ne + e], l = b.lL1[e];
    acc += 3.0 * wtd(i) * (cx(i) * (ok ? gx : 0.0) + cy(i) * (ok ? gy : 0.0));
    acc += 6.0 * wtd(i) * (ok ? l : 0.0);
  }
  if (in1) {
    const int e = i1(g, zx, zy);
    acc += -6.0 * (1.0 - wtd(0)) * b.lL1[e] + b.lphie1[e];
  }
  b.lphie2[k] = acc;
}

// Interior: fold the e2 adjoint of phi back (transpose of the extension) and
// add it to every h_i (phi = sum_i h_i); write lambda_n.
__global__ __launch_bounds__(kB) void k_adj_b7(AGrid g, ABuf b, double* __restrict__ lam_out) {
  const int N = g.nx * g.ny;
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  const int x = k % g.nx, y = k / g.nx;
  double lphi = b.lphi[k];
  int px[3], rx[3], py[3], ry[3];
  const int mx = preimages(x, g.nx, g.wx, 2, px, rx), my = preimages(y, g.ny, g.wy, 2, py, ry);
  for (int a = 0; a < mx; ++a)
    for (int bb = 0; bb < my; ++bb) lphi += b.lphie2[i2(g, px[a], py[bb])];
  for (int i = 0; i < 9; ++i) {
    lam_out[(size_t)i * N + k] = b.lf[(size_t)i * N + k];
    lam_out[(size_t)(9 + i) * N + k] = b.lh[(size_t)i * N + k] + lphi;
  }
}

__global__ __launch_bounds__(kB) void k_adj_fa_init(AGrid g, const float* __restrict__ phi0, double* __restrict__ phie2) {
  const int ne = (g.nx + 4) * (g.ny + 4);
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= ne) return;
  const int ex = k % (g.nx + 4) - 2, ey = k / (g.nx + 4) - 2;
  int r;
  const int x = ext_map(ex, g.nx, g.wx, r), y = ext_map(ey, g.ny, g.wy, r);
  phie2[k] = (double)phi0[i0(g, x, y)];
}

// Adjoint of the initial state (A11): f = f^eq(0, rho(phi0), u0),
// h = h^eq(phi0, mu(phi0), u0), J = phi0 u0.  Step 1: node-local part.
__global__ __launch_bounds__(kB) void k_adj_init_a(AGrid g, ACon c, ABuf b, const float* __restrict__ phi0, const float* __restrict__ ux0,
                             const float* __restrict__ uy0, const double* __restrict__ lam) {
  const int N = g.nx * g.ny, ne = (g.nx + 2) * (g.ny + 2);
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= ne) return;
  const int ex = k % (g.nx + 2) - 1, ey = k / (g.nx + 2) - 1;
  if (ex < 0 || ex >= g.nx || ey < 0 || ey >= g.ny) return;
  const int n = i0(g, ex, ey);
  const double p = phi0[n], ux = ux0 ? ux0[n] : 0.0, uy = uy0 ? uy0[n] : 0.0;
  const double usq = ux * ux + uy * uy;
  double lrho = 0, lphi = 0, lmu = 0;
  for (int i = 0; i < 9; ++i) {
    const double cu = cx(i) * ux + cy(i) * uy;
    const double si = 3.0 * cu + 4.5 * cu * cu - 1.5 * usq;
    lrho += wtd(i) * CS2 * si * lam[(size_t)i * N + n];
    const double lh = lam[(size_t)(9 + i) * N + n];
    if (i == 0) { lphi += lh; lmu += (wtd(0) - 1.0) * lh; }
    else { lphi += 3.0 * wtd(i) * cu * lh; lmu += wtd(i) * lh; }
  }
  lphi += ux * lam[(size_t)18 * N + n] + uy * lam[(size_t)19 * N + n];
  lphi += c.drho_h * lrho;
  b.lphi[n] = lphi;
  b.lmun[n] = lmu;   // sum_i wbar'_i lambda_h_i (h^eq depends on eta mu)
}

// Step 2 (e1 grid first ring + interior): mu0 = 4 beta phi (phi^2-1) - kappa lap(phi0_e1)
__global__ __launch_bounds__(kB) void k_adj_init_b(AGrid g, ACon c, ABuf b) {
  const int ne = (g.nx + 2) * (g.ny + 2);
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= ne) return;
  const int ex = k % (g.nx + 2) - 1, ey = k / (g.nx + 2) - 1;
  const bool in = ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny;
  const double sw = in ? b.lmun[i0(g, ex, ey)] : 0.0;
  const double lmu = c.eta * sw;
  const double p = b.phie2[i2(g, ex, ey)];
  double l = 0;
  if (in)
    for (int i = 1; i < 9; ++i) l += wtd(i) * (b.phie2[i2(g, ex + cx(i), ey + cy(i))] - p);
  const double mu = c.beta4 * p * (p * p - 1.0) - c.kappa * 6.0 * l;
  if (in) {
    b.gsig[k] += lmu * mu / c.sigma;
    b.gM[k] += sw * mu * c.detadM;
  }
  b.lL1[k] = in ? -c.kappa * lmu : 0.0;
  b.lphie1[k] = in ? c.beta4 * (3.0 * p * p - 1.0) * lmu : 0.0;
  b.lG1[k] = 0.0;
  b.lG1[ne + k] = 0.0;
}

// Step 3: transposed Laplacian onto e1 positions, folded onto the nodes.
__global__ __launch_bounds__(kB) void k_adj_init_c(AGrid g, ABuf b, double* __restrict__ dphi0) {
  const int N = g.nx * g.ny;
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  const int x = k % g.nx, y = k / g.nx;
  double acc = b.lphi[k];
  int px[3], rx[3], py[3], ry[3];
  const int mx = preimages(x, g.nx, g.wx, 1, px, rx), my = preimages(y, g.ny, g.wy, 1, py, ry);
  for (int a = 0; a < mx; ++a)
    for (int bb = 0; bb < my; ++bb) {
      const int zx = px[a], zy = py[bb];
      double s = 0;
      for (int i = 1; i < 9; ++i) {
        const int ex = zx - cx(i), ey = zy - cy(i);
        if (ex < 0 || ex >= g.nx || ey < 0 || ey >= g.ny) continue;   // lap taken at nodes only
        s += 6.0 * wtd(i) * b.lL1[i1(g, ex, ey)];
      }
      if (zx >= 0 && zx < g.nx && zy >= 0 && zy < g.ny) s += -6.0 * (1.0 - wtd(0)) * b.lL1[i1(g, zx, zy)] + b.lphie1[i1(g, zx, zy)];
      acc += s;
    }
  dphi0[k] = acc;
}

__global__ __launch_bounds__(kB) void k_adj_zero(double* p, long long n) {
  const long long k = (long long)blockIdx.x * kB + threadIdx.x;
  if (k < n) p[k] = 0.0;
}

__global__ __launch_bounds__(kB) void k_adj_sum(const double* __restrict__ a, long long n, double* out) {   // one block
  __shared__ double red[kB];
  double s = 0;
  for (long long k = threadIdx.x; k < n; k += kB) s += a[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ __launch_bounds__(kB) void k_adj_seed(AGrid g, const double* __restrict__ phi, const float* __restrict__ target,
                           double* __restrict__ lam, double* __restrict__ lossd) {
  const int N = g.nx * g.ny;
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  const double r = phi[k] - (double)target[k];
  for (int i = 0; i < 9; ++i) {
    lam[(size_t)i * N + k] = 0.0;
    lam[(size_t)(9 + i) * N + k] = r;   // phi = sum_i h_i
  }
  lam[(size_t)18 * N + k] = 0.0;
  lam[(size_t)19 * N + k] = 0.0;
  lossd[k] = 0.5 * r * r;
}

unsigned nblk(long long n) { return (unsigned)((n + kB - 1) / kB); }

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct lbm_adj {
  lbm_sim* sim;
  lbm_params p;
  AGrid g;
  ACon c;
  ABuf b;
  char* ws;
  double* red;   // two doubles + loss
  double* lossd;
};

namespace {

struct AdjLayout {
  size_t total;
  std::vector<std::pair<double**, size_t>> items;
};

size_t adj_doubles(const lbm_params* p) {
  const size_t N = (size_t)p->nx * p->ny, N1 = (size_t)(p->nx + 2) * (p->ny + 2),
               N2 = (size_t)(p->nx + 4) * (p->ny + 4);
  // interior planes: f9 h9 J2 phi Fsf2 F2 rho muv tauf u2 gr2 P Q2 D dQ2 divn lf9 lh9 lP lrho lu2 lF2 lgr2 lphi lD lQ2
  //                  lmun lossd
  const size_t nin = 9 + 9 + 2 + 1 + 2 + 2 + 1 + 1 + 1 + 2 + 2 + 1 + 2 + 1 + 2 + 1 + 9 + 9 + 1 + 1 + 2 + 2 + 2 + 1 +
                     1 + 2 + 1 + 1;
  // e1 planes: G1 2, L1, mu1, T1 3, n1 2, s1, ue1 2, Q1 2, lue1 2, lphie1, lG1 2, lL1, gsig, gM
  const size_t ne1 = 2 + 1 + 1 + 3 + 2 + 1 + 2 + 2 + 2 + 1 + 2 + 1 + 1 + 1;
  // e2 planes: phie2, lphie2
  return nin * N + ne1 * N1 + 2 * N2 + 8;
}

}  // namespace

extern "C" {

int lbm_adjoint_workspace_bytes(const lbm_params* p, size_t* bytes) {
  size_t dummy;
  if (int r = lbm_workspace_bytes(p, &dummy)) return r;
  if (!bytes) return set_error(LBM_E_INVAL, "bytes is NULL");
  *bytes = adj_doubles(p) * sizeof(double) + 4096;
  return LBM_OK;
}

int lbm_adjoint_create(lbm_adj** out, lbm_sim* sim, void* d_ws, size_t ws_bytes) {
  if (!out || !sim || !d_ws) return set_error(LBM_E_INVAL, "NULL argument");
  *out = nullptr;
  lbm_params p;
  if (int r = sim_params(sim, &p)) return r;
  size_t need = 0;
  if (int r = lbm_adjoint_workspace_bytes(&p, &need)) return r;
  if (ws_bytes < need) return set_error(LBM_E_INVAL, "adjoint workspace too small: %zu < %zu", ws_bytes, need);
  if (((uintptr_t)d_ws % 256) != 0) return set_error(LBM_E_INVAL, "workspace must be 256-byte aligned");
  if (!(p.sigma > 0)) return set_error(LBM_E_INVAL, "the adjoint needs sigma > 0");
  lbm_adj* a = new (std::nothrow) lbm_adj();
  if (!a) return set_error(LBM_E_INVAL, "out of host memory");
  a->sim = sim;
  a->p = p;
  a->ws = (char*)d_ws;
  const int nx = p.nx, ny = p.ny;
  if (p.wall_x == 2 || p.wall_y == 2) {
    delete a;
    return set_error(LBM_E_UNSUPPORTED, "the adjoint supports periodic and no-slip walls only");
  }
  a->g.nx = nx; a->g.ny = ny; a->g.wx = p.wall_x; a->g.wy = p.wall_y;
  {
    SimView v;
    if (int r = sim_view(sim, &v)) { delete a; return r; }
    a->g.sg = v.g;
  }
  const Phys ph = sim_phys(sim);
  ACon& c = a->c;
  c.beta4 = ph.beta4_d; c.kappa = ph.kappa_d; c.sigma = p.sigma; c.eps2 = ph.eps2_d;
  c.eta = ph.eta_d; c.detadM = 1.0 / (CS2 * (p.tau_h - 0.5)); c.a_h = ph.a_h_d; c.inv_tau_h = ph.inv_tau_h_d;
  c.rho2 = ph.rho2_d; c.drho_h = ph.drho_half_d; c.mu2 = ph.mu2_d; c.dmu_h = ph.dmu_half_d;
  c.gx = ph.gx_d; c.gy = ph.gy_d; c.rho0 = ph.rho0_d; c.uw_lo = ph.uw_lo_d; c.uw_hi = ph.uw_hi_d;
  c.form = 0;
  const size_t N = (size_t)nx * ny, N1 = (size_t)(nx + 2) * (ny + 2), N2 = (size_t)(nx + 4) * (ny + 4);
  double* q = (double*)d_ws;
  auto take = [&](size_t n) { double* r = q; q += n; return r; };
  ABuf& b = a->b;
  b.f = take(9 * N); b.h = take(9 * N); b.J = take(2 * N); b.phi = take(N);
  b.Fsf = take(2 * N); b.F = take(2 * N); b.rho = take(N); b.muv = take(N); b.tauf = take(N); b.u = take(2 * N);
  b.gr = take(2 * N); b.P = take(N); b.Q = take(2 * N); b.D = take(N); b.dQ = take(2 * N); b.divn = take(N);
  b.lf = take(9 * N); b.lh = take(9 * N); b.lP = take(N); b.lrho = take(N); b.lu = take(2 * N); b.lF = take(2 * N);
  b.lgr = take(2 * N); b.lphi = take(N); b.lD = take(N); b.lQ = take(2 * N); b.lmun = take(N);
  a->lossd = take(N);
  b.G1 = take(2 * N1); b.L1 = take(N1); b.mu1 = take(N1); b.T1 = take(3 * N1); b.n1 = take(2 * N1); b.s1 = take(N1);
  b.ue1 = take(2 * N1); b.Q1 = take(2 * N1); b.lue1 = take(2 * N1); b.lphie1 = take(N1);
  b.lG1 = take(2 * N1); b.lL1 = take(N1); b.gsig = take(N1); b.gM = take(N1);
  b.phie2 = take(N2); b.lphie2 = take(N2);
  a->red = take(8);
  *out = a;
  return lbm_adjoint_reset(a, nullptr);
}

int lbm_adjoint_reset(lbm_adj* a, void* stream) {
  if (!a) return set_error(LBM_E_INVAL, "adjoint is NULL");
  const size_t N1 = (size_t)(a->p.nx + 2) * (a->p.ny + 2);
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_adj_zero, dim3(nblk(N1)), dim3(kB), 0, st, a->b.gsig, (long long)N1);
  hipLaunchKernelGGL(k_adj_zero, dim3(nblk(N1)), dim3(kB), 0, st, a->b.gM, (long long)N1);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LBM_OK : set_error(LBM_E_HIP, "adjoint reset: %s", hipGetErrorString(e));
}

int lbm_adjoint_seed_phi_misfit(lbm_adj* a, const float* d_target, double* d_lambda, double* h_loss, void* stream) {
  if (!a || !d_target || !d_lambda) return set_error(LBM_E_INVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  const size_t N = (size_t)a->p.nx * a->p.ny;
  SimView v;
  if (int r = sim_view(a->sim, &v)) return r;
  hipLaunchKernelGGL(k_adj_unpack, dim3(nblk(N)), dim3(kB), 0, st, v.s, v.phi, a->g, a->b);
  hipLaunchKernelGGL(k_adj_fa, dim3(nblk((a->p.nx + 4) * (a->p.ny + 4))), dim3(kB), 0, st, a->g, a->b);
  hipLaunchKernelGGL(k_adj_seed, dim3(nblk(N)), dim3(kB), 0, st, a->g, a->b.phi, d_target, d_lambda, a->lossd);
  hipLaunchKernelGGL(k_adj_sum, dim3(1), dim3(kB), 0, st, a->lossd, (long long)N, a->red + 2);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && h_loss) {
    e = hipMemcpyAsync(h_loss, a->red + 2, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  return e == hipSuccess ? LBM_OK : set_error(LBM_E_HIP, "adjoint seed: %s", hipGetErrorString(e));
}

namespace {

// One adjoint step linearised about the state (S, phi).  lambda is updated in
// place: k_adj_b1 is the only reader of its planes 0-17 (at neighbouring
// nodes) and reads planes 18-19 of its own node before writing them;
// k_adj_b7 writes planes 0-17 after b1 has finished.
int adjoint_step_at(lbm_adj* a, const float* S, const double* phis, int32_t form, double* d_lambda, hipStream_t st) {
  a->c.form = form;
  const AGrid& g = a->g;
  const long long N = (long long)g.nx * g.ny, N1 = (long long)(g.nx + 2) * (g.ny + 2),
                  N2 = (long long)(g.nx + 4) * (g.ny + 4);
  hipLaunchKernelGGL(k_adj_unpack, dim3(nblk(N)), dim3(kB), 0, st, S, phis, g, a->b);
  hipLaunchKernelGGL(k_adj_fa, dim3(nblk(N2)), dim3(kB), 0, st, g, a->b);
  hipLaunchKernelGGL(k_adj_fb, dim3(nblk(N1)), dim3(kB), 0, st, g, a->c, a->b);
  hipLaunchKernelGGL(k_adj_fc, dim3(nblk(N)), dim3(kB), 0, st, g, a->c, a->b);
  hipLaunchKernelGGL(k_adj_fd, dim3(nblk(N1)), dim3(kB), 0, st, g, a->c, a->b);
  hipLaunchKernelGGL(k_adj_fe, dim3(nblk(N)), dim3(kB), 0, st, g, a->b);
  hipLaunchKernelGGL(k_adj_b1, dim3(nblk(N)), dim3(kB), 0, st, g, a->c, a->b, d_lambda, d_lambda);
  hipLaunchKernelGGL(k_adj_b2, dim3(nblk(N1)), dim3(kB), 0, st, g, a->b);
  hipLaunchKernelGGL(k_adj_b3, dim3(nblk(N)), dim3(kB), 0, st, g, a->c, a->b);
  hipLaunchKernelGGL(k_adj_b4, dim3(nblk(N1)), dim3(kB), 0, st, g, a->c, a->b);
  hipLaunchKernelGGL(k_adj_b6, dim3(nblk(N2)), dim3(kB), 0, st, g, a->b);
  hipLaunchKernelGGL(k_adj_b7, dim3(nblk(N)), dim3(kB), 0, st, g, a->b, d_lambda);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LBM_OK : set_error(LBM_E_HIP, "adjoint step: %s", hipGetErrorString(e));
}

}  // namespace

int lbm_adjoint_step(lbm_adj* a, int32_t form, double* d_lambda, void* stream) {
  if (!a || !d_lambda) return set_error(LBM_E_INVAL, "NULL argument");
  if (form < 0 || form >= LBM_NUM_FORMS) return set_error(LBM_E_INVAL, "bad force form %d", form);
  SimView v;
  if (int r = sim_view(a->sim, &v)) return r;
  return adjoint_step_at(a, v.s, v.phi, form, d_lambda, (hipStream_t)stream);
}

int lbm_adjoint_step_blob(lbm_adj* a, const void* d_blob, int32_t form, double* d_lambda, void* stream) {
  if (!a || !d_blob || !d_lambda) return set_error(LBM_E_INVAL, "NULL argument");
  if (form < 0 || form >= LBM_NUM_FORMS) return set_error(LBM_E_INVAL, "bad force form %d", form);
  SimView v;
  if (int r = sim_view(a->sim, &v)) return r;
  const char* b = (const char*)d_blob;   // lbm_save layout: state array, then phi
  const size_t sb = (size_t)kNPL * (size_t)v.g.ps * sizeof(float);
  return adjoint_step_at(a, (const float*)b, (const double*)(b + sb), form, d_lambda, (hipStream_t)stream);
}

int lbm_adjoint_init(lbm_adj* a, const float* d_phi0, const float* d_ux0, const float* d_uy0, const double* d_lambda0,
                     double* d_dphi0, void* stream) {
  if (!a || !d_phi0 || !d_lambda0 || !d_dphi0) return set_error(LBM_E_INVAL, "NULL argument");
  if ((d_ux0 == nullptr) != (d_uy0 == nullptr)) return set_error(LBM_E_INVAL, "give both u0 components or neither");
  hipStream_t st = (hipStream_t)stream;
  const AGrid& g = a->g;
  const long long N = (long long)g.nx * g.ny, N1 = (long long)(g.nx + 2) * (g.ny + 2);
  hipLaunchKernelGGL(k_adj_fa_init, dim3(nblk((long long)(g.nx + 4) * (g.ny + 4))), dim3(kB), 0, st, g, d_phi0,
                     a->b.phie2);
  hipLaunchKernelGGL(k_adj_init_a, dim3(nblk(N1)), dim3(kB), 0, st, g, a->c, a->b, d_phi0, d_ux0, d_uy0, d_lambda0);
  hipLaunchKernelGGL(k_adj_init_b, dim3(nblk(N1)), dim3(kB), 0, st, g, a->c, a->b);
  hipLaunchKernelGGL(k_adj_init_c, dim3(nblk(N)), dim3(kB), 0, st, g, a->b, d_dphi0);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LBM_OK : set_error(LBM_E_HIP, "adjoint init: %s", hipGetErrorString(e));
}

int lbm_adjoint_param_grads(lbm_adj* a, double* h_dsigma, double* h_dM, void* stream) {
  if (!a || !h_dsigma || !h_dM) return set_error(LBM_E_INVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  const long long N1 = (long long)(a->p.nx + 2) * (a->p.ny + 2);
  hipLaunchKernelGGL(k_adj_sum, dim3(1), dim3(kB), 0, st, a->b.gsig, N1, a->red);
  hipLaunchKernelGGL(k_adj_sum, dim3(1), dim3(kB), 0, st, a->b.gM, N1, a->red + 1);
  double h[2];
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(h, a->red, 2 * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return set_error(LBM_E_HIP, "adjoint grads: %s", hipGetErrorString(e));
  *h_dsigma = h[0];
  *h_dM = h[1];
  return LBM_OK;
}

int lbm_adjoint_destroy(lbm_adj* a) {
  delete a;
  return LBM_OK;
}

}  // extern "C"
