// Hand-written adjoint of one time step of the phase-field LBM
// (arXiv:2012.14729, Sec. II-IV), and of the initial state.
//
// The adjoint acts on the physical pre-collision state of a step: f_i, h_i
// (i = 0..8) and J = (phi u) of the previous step, nine + nine + two FP64
// values per node.  Given lambda_{n+1} = dL/ds_{n+1} it returns
// lambda_n = (ds_{n+1}/ds_n)^T lambda_{n+1} in a second array, and adds the
// step's terms of dL/dsigma and dL/dM to per-tile accumulators.
//
// Two kernels per adjoint step, both on 32x8-node tiles (one node per
// thread) with the order parameter staged in LDS like the step kernels:
//   k_adj_a  recomputes the forward quantities of each node from the saved
//            state (phi stencils, F_sf, u, P; the shared tile code of
//            lbm_tile.hpp), gathers lambda_{n+1} along the streamed links
//            (bounce-back at walls, Eq. 43) and transposes both collisions
//            (Eqs. 29-36).  It writes the node-level adjoints of D =
//            div(phi u), u, rho, F, grad rho, phi, mu and P (plus u and F_sf)
//            to a scratch array, and the J part of lambda_n.
//   k_adj_b  transposes what couples nodes: div(phi u) with the ghost
//            velocity of Sec. IV (reading A9), u = (j + F/2)/rho, the force
//            form's stencils (Sec. II.B), mu_phi (Eq. 2), grad rho, and the
//            gradient and Laplacian of phi (Eqs. 41-42) with the even
//            reflection of phi at walls; ghost contributions fold back onto
//            their mirror nodes.  It writes the f and h parts of lambda_n.
// A tile of k_adj_b works on an LDS window around it: phi with 4 halo nodes,
// grad/lap phi and the adjoint of D with 3, the adjoint of F with 2 and the
// adjoints of grad/lap/mu with 1, so every sum it takes is a plain gather.
// All arithmetic is FP64; the gradients of sigma and M are summed per tile
// in a fixed order, so the results are deterministic.
#include <cmath>
#include <cstdint>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_tile.hpp"

namespace pflbm {

namespace {

constexpr double kC2 = 1.0 / 3.0;   // cs^2
using AS = Shape<32, 8>;            // adjoint tile: 32 x 8 nodes, 256 threads
constexpr int kAT = AS::NT;
constexpr int kB = 256;             // node-parallel kernels (init, seed, sums)
constexpr int kRed = 256;           // partial sums of a reduction

struct ACon {
  double beta4, kappa, sigma, eps2, eta, detadM, a_h, inv_tau_h;
  double rho2, drho_h, mu2, dmu_h, gx, gy, rho0, uw_lo, uw_hi;
};

// Scratch planes written by k_adj_a (dense row-major [ny][nx], FP64): the
// adjoints of D, u (2), rho, F (2), grad rho (2), phi, mu (through h^eq) and
// P at each node, and the node's u (2) and F_sf (2).
enum : int { kSD, kSUX, kSUY, kSRHO, kSFX, kSFY, kSGX, kSGY, kSPHI, kSMU, kSP, kSVX, kSVY, kSFSX, kSFSY, kNS };

struct AArgs {
  StepArgs a;          // sin: saved state array; phi: saved FP64 phi plane; g, c
  const double* lin;   // lambda_{n+1}: 20 planes [ny][nx] (f 0-8, h 9-17, J 18-19)
  double* lout;        // lambda_n (distinct from lin)
  double* scr;         // kNS planes
  double* gsig;        // per-tile dL/dsigma terms [ntiles]
  double* gM;          // per-tile dL/dM terms [ntiles]
  ACon c;
  int nx, ny, wx, wy;
};

struct AGrid {
  int nx, ny, wx, wy;
};

__device__ __forceinline__ int i0(const AGrid& g, int x, int y) { return y * g.nx + x; }
__device__ __forceinline__ int i1(const AGrid& g, int x, int y) { return (y + 1) * (g.nx + 2) + (x + 1); }
__device__ __forceinline__ int i2(const AGrid& g, int x, int y) { return (y + 2) * (g.nx + 4) + (x + 2); }

// extension map along one axis: position p in [-k, n+k) -> node, with a
// reflection flag (even reflection about a half-way wall, Sec. IV)
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

// Deterministic sum over a workgroup of kAT threads (wave reduction, then the
// four wave sums in order); the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kAT / 64; ++k) s += red[k];
  return s;
}

// ---------------------------------------------------------------------------
// k_adj_a: forward recomputation and the transposes of streaming and of the
// two collisions, node-local after the gather of lambda_{n+1}.
// ---------------------------------------------------------------------------
template <int FORM, int BC>
__global__ __launch_bounds__(kAT) void k_adj_a(AArgs A) {
  __shared__ Lds<AS> s;
  __shared__ double red[kAT / 64];
  constexpr bool WX = (BC & 1) != 0, WY = (BC & 2) != 0;
  const int ntx = (A.nx + AS::TX - 1) / AS::TX, nty = (A.ny + AS::TY - 1) / AS::TY;
  int tile_x, tile_y;
  if (!xcd_tile(ntx, nty, tile_x, tile_y)) return;
  const StepArgs& a = A.a;
  const Phys& c = a.c;
  const ACon& C = A.c;
  const int tid = threadIdx.x;
  constexpr int PW = AS::PW, PH = AS::PH;
  const int x0 = tile_x * AS::TX, y0 = tile_y * AS::TY;
  const int lx = tid & (AS::TX - 1), ty = tid / AS::TX;
  const int x = x0 + lx, y = y0 + ty;
  const bool act = x < A.nx && y < A.ny;
  // phi with a 3-node halo (periodic wrap / even reflection, Sec. IV)
  for (int k = tid; k < PH * PW; k += kAT) {
    const int py = k / PW, px = k - py * PW;
    s.phi[py][px] = a.phi[(unsigned)(halo_coord<WY>(y0 + py - 3, A.ny) * a.g.pitch + halo_coord<WX>(x0 + px - 3, A.nx))];
  }
  __syncthreads();
  stage_b<FORM, AS>(s, tid, c);
  __syncthreads();
  double dM = 0.0;
  if (act) {
    const int N = A.nx * A.ny, k = y * A.nx + x;
    float ft[9];
    load_fp<WX, WY>(a, x, y, ft);
    // lambda_{n+1} along the streamed links: the post-collision value of
    // direction i at x became population i at x + c_i, or population opp(i)
    // at x where x + c_i lies beyond a wall (Eq. 43)
    double lfp[9], lhp[9], cuw[9];
    bool hit[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      int tx = x + cx(i), tyy = y + cy(i);
      bool h = false;
      double cw = 0.0;
      if (tx < 0 || tx >= A.nx) {
        if (WX) { h = true; cw = cy(i) * (tx < 0 ? C.uw_lo : C.uw_hi); }
        else tx = tx < 0 ? tx + A.nx : tx - A.nx;
      }
      if (tyy < 0 || tyy >= A.ny) {
        if (WY) { h = true; cw = cx(i) * (tyy < 0 ? C.uw_lo : C.uw_hi); }
        else tyy = tyy < 0 ? tyy + A.ny : tyy - A.ny;
      }
      const int slot = h ? opp(i) : i;
      const int tgt = h ? k : tyy * A.nx + tx;
      hit[i] = h;
      cuw[i] = cw;
      lfp[i] = A.lin[(size_t)slot * N + tgt];
      lhp[i] = A.lin[(size_t)(9 + slot) * N + tgt];
    }
    const double lJx = A.lin[(size_t)18 * N + k], lJy = A.lin[(size_t)19 * N + k];
    // forward quantities of the node (Sec. II.B, Eqs. 8-10, 37, reading A6)
    double fsx, fsy;
    force_sf<FORM, AS>(s, ty + 1, lx + 1, c, fsx, fsy);
    const double phi = s.phi[ty + 3][lx + 3];
    const double gxp = s.gl[0][ty + 2][lx + 2], gyp = s.gl[1][ty + 2][lx + 2], lap = s.gl[2][ty + 2][lx + 2];
    const double mu = chem_pot(phi, lap, c);
    const double rho = rho_of(phi, c), muv = mu_of(phi, c);
    const double Fx = fsx + (rho - C.rho0) * C.gx, Fy = fsy + (rho - C.rho0) * C.gy;
    double fv[9], jx = 0.0, jy = 0.0, S = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      fv[i] = (double)ft[i];
      jx += cx(i) * fv[i];
      jy += cy(i) * fv[i];
      S += fv[i];
    }
    const double ux = (jx + 0.5 * kC2 * Fx) / (kC2 * rho), uy = (jy + 0.5 * kC2 * Fy) / (kC2 * rho);
    const double grx = C.drho_h * gxp, gry = C.drho_h * gyp;
    const double P = S + 0.5 * kC2 * (ux * grx + uy * gry);
    const double tauf = 0.5 + muv / (kC2 * rho);
    const double om = 1.0 / tauf, cf = 1.0 - 0.5 * om, omh = C.inv_tau_h, cfh = 1.0 - 0.5 * omh;
    const double usq = ux * ux + uy * uy;
    double lP = 0, lrho = 0, lux = 0, luy = 0, lFx = 0, lFy = 0, lgx = 0, lgy = 0, lphi = 0, lmu = 0, lD = 0;
    double ldqx = 0, ldqy = 0, lom = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      if (hit[i]) {   // f_opp = f_i^+ - 2 w_i rho c_i.u_w ; h_opp = h_i^+ - 6 w_i phi c_i.u_w
        lrho += -2.0 * wtd(i) * cuw[i] * lfp[i];
        lphi += -6.0 * wtd(i) * cuw[i] * lhp[i];
      }
      // flow collision f^+ = (1 - om) f + om feq + cf F_i   (Eqs. 29, 31, 35, reading A1)
      const double cu = cx(i) * ux + cy(i) * uy;
      const double si = 3.0 * cu + 4.5 * cu * cu - 1.5 * usq;
      const double feq = wtd(i) * (P + kC2 * rho * si);
      const double Vx = wtd(i) * (1.0 + si) * Fx + wtd(i) * si * kC2 * grx;
      const double Vy = wtd(i) * (1.0 + si) * Fy + wtd(i) * si * kC2 * gry;
      const double Fi = (cx(i) - ux) * Vx + (cy(i) - uy) * Vy;
      lom += lfp[i] * (feq - fv[i] - 0.5 * Fi);
      const double lfeq = om * lfp[i], lFi = cf * lfp[i];
      lP += wtd(i) * lfeq;
      lrho += wtd(i) * kC2 * si * lfeq;
      double lsi = wtd(i) * kC2 * rho * lfeq;
      lux += -Vx * lFi;
      luy += -Vy * lFi;
      const double lVx = (cx(i) - ux) * lFi, lVy = (cy(i) - uy) * lFi;
      lFx += wtd(i) * (1.0 + si) * lVx;
      lFy += wtd(i) * (1.0 + si) * lVy;
      lgx += wtd(i) * si * kC2 * lVx;
      lgy += wtd(i) * si * kC2 * lVy;
      lsi += wtd(i) * (Fx * lVx + Fy * lVy) + wtd(i) * kC2 * (grx * lVx + gry * lVy);
      lux += lsi * (3.0 * cx(i) + 9.0 * cu * cx(i) - 3.0 * ux);
      luy += lsi * (3.0 * cy(i) + 9.0 * cu * cy(i) - 3.0 * uy);
      // order-parameter collision h^+ = (1 - omh) h + omh heq + cfh H_i   (Eqs. 30, 32, 36)
      const double lheq = omh * lhp[i], lH = cfh * lhp[i];
      const double wb = i == 0 ? wtd(0) - 1.0 : wtd(i);
      if (i == 0) {
        lphi += lheq;
      } else {
        lphi += 3.0 * wtd(i) * cu * lheq;
        lux += 3.0 * wtd(i) * phi * cx(i) * lheq;
        luy += 3.0 * wtd(i) * phi * cy(i) * lheq;
      }
      lmu += C.eta * wb * lheq;
      dM += mu * wb * lheq * C.detadM;
      lD += wb * C.a_h * lH;
      ldqx += 3.0 * wtd(i) * cx(i) * lH;
      ldqy += 3.0 * wtd(i) * cy(i) * lH;
    }
    // tau_f = 1/2 + mu/(cs^2 rho), om = 1/tau_f   (A6)
    const double ltau = -lom / (tauf * tauf);
    lrho += -muv / (kC2 * rho * rho) * ltau;
    lphi += C.dmu_h * ltau / (kC2 * rho);
    // P = S + cs^2/2 u.grad rho   (Eq. 37)
    lux += 0.5 * kC2 * grx * lP;
    luy += 0.5 * kC2 * gry * lP;
    lgx += 0.5 * kC2 * ux * lP;
    lgy += 0.5 * kC2 * uy * lP;
    // J_{n+1} = Q, d_t Q = Q - J_n (A4), Q = phi u at the node; the part of
    // the adjoint of Q that div(phi u) carries from the neighbours is added
    // by k_adj_b
    const double lQx = lJx + ldqx, lQy = lJy + ldqy;
    A.lout[(size_t)18 * N + k] = -ldqx;
    A.lout[(size_t)19 * N + k] = -ldqy;
    lux += phi * lQx;
    luy += phi * lQy;
    lphi += ux * lQx + uy * lQy;
    double* sc = A.scr;
    sc[(size_t)kSD * N + k] = lD;
    sc[(size_t)kSUX * N + k] = lux;
    sc[(size_t)kSUY * N + k] = luy;
    sc[(size_t)kSRHO * N + k] = lrho;
    sc[(size_t)kSFX * N + k] = lFx;
    sc[(size_t)kSFY * N + k] = lFy;
    sc[(size_t)kSGX * N + k] = lgx;
    sc[(size_t)kSGY * N + k] = lgy;
    sc[(size_t)kSPHI * N + k] = lphi;
    sc[(size_t)kSMU * N + k] = lmu;
    sc[(size_t)kSP * N + k] = lP;
    sc[(size_t)kSVX * N + k] = ux;
    sc[(size_t)kSVY * N + k] = uy;
    sc[(size_t)kSFSX * N + k] = fsx;
    sc[(size_t)kSFSY * N + k] = fsy;
  }
  const double tot = block_sum(dM, red);
  if (tid == 0) A.gM[tile_y * ntx + tile_x] += tot;
}

// ---------------------------------------------------------------------------
// k_adj_b: the transposes that couple nodes, on an LDS window around the tile.
// ---------------------------------------------------------------------------
constexpr int kH4W = AS::TX + 8, kH4H = AS::TY + 8;   // halo 4
constexpr int kH3W = AS::TX + 6, kH3H = AS::TY + 6;   // halo 3
constexpr int kH2W = AS::TX + 4, kH2H = AS::TY + 4;   // halo 2
constexpr int kH1W = AS::TX + 2, kH1H = AS::TY + 2;   // halo 1

// ld lives in phases 0-1 and la in phases 3-4, so they share storage: the
// window then takes 51 KB, and two workgroups leave room on a CU for a
// 512-thread step kernel from another stream (the overlapped recompute).
struct AdjLds {
  double phi[kH4H][kH4W];       // phi extended (wrap / even reflection)
  double gl[3][kH3H][kH3W];     // grad phi (x, y), lap phi
  union {
    double ld[kH3H][kH3W];      // adjoint of D = div(phi u) at nodes (0 beyond walls)
    double la[4][kH1H][kH1W];   // adjoints of grad phi (2), lap phi, and the phi part of mu_phi
  };
  double lq[2][kH3H][kH3W];     // adjoint of the extended node field phi u, from div
  double lf[3][kH2H][kH2W];     // adjoint of F_sf at nodes (2) and, for CSF, of div n
  double lp[kH2H][kH2W];        // adjoint of the extended phi from the stencils and mu_phi
  double red[kAT / 64];
};

// Window position (px, py), relative to the tile origin, to a node: true and
// the node's dense index when it lies inside the domain (periodic axes wrap).
__device__ __forceinline__ bool window_node(int gx, int gy, const AArgs& A, int& k) {
  if (gx < 0 || gx >= A.nx) {
    if (A.wx) return false;
    gx = gx < 0 ? gx + A.nx : gx - A.nx;
  }
  if (gy < 0 || gy >= A.ny) {
    if (A.wy) return false;
    gy = gy < 0 ? gy + A.ny : gy - A.ny;
  }
  k = gy * A.nx + gx;
  return true;
}

// Image positions of node (gx, gy) one step beyond a wall (the ghost
// positions whose velocity and phi u are built from this node, reading A9),
// as window offsets with their reflection flags; returns the count (<= 4,
// the node itself first).
__device__ __forceinline__ int ghost_images(int gx, int gy, const AArgs& A, int* dx, int* dy, int* rx, int* ry) {
  int ox[2] = {0, 0}, oxr[2] = {0, 0}, nx_ = 1, oy[2] = {0, 0}, oyr[2] = {0, 0}, ny_ = 1;
  if (A.wx) {
    if (gx == 0) { ox[nx_] = -1; oxr[nx_] = 1; ++nx_; }
    else if (gx == A.nx - 1) { ox[nx_] = 1; oxr[nx_] = 1; ++nx_; }
  }
  if (A.wy) {
    if (gy == 0) { oy[ny_] = -1; oyr[ny_] = 1; ++ny_; }
    else if (gy == A.ny - 1) { oy[ny_] = 1; oyr[ny_] = 1; ++ny_; }
  }
  int m = 0;
  for (int a = 0; a < nx_; ++a)
    for (int b = 0; b < ny_; ++b) {
      dx[m] = ox[a]; rx[m] = oxr[a];
      dy[m] = oy[b]; ry[m] = oyr[b];
      ++m;
    }
  return m;
}

// Adjoint of u at node (gx, gy), window position (px, py): the node's own
// part (lu) plus the part that div(phi u) carries through the node's phi u
// and through the ghost velocities built from it (u_ghost = 2 u_w - u at a
// no-slip wall, both components flipped); also returns the adjoint of phi
// from those same terms (phi of a ghost is the mirror node's, and its phi u
// carries the wall velocity).
__device__ __forceinline__ void u_adjoint(const AdjLds& L, const AArgs& A, int px, int py, int gx, int gy, double ux,
                                          double uy, double phi, double lux0, double luy0, double& lux, double& luy,
                                          double& lphi) {
  int dx[4], dy[4], rx[4], ry[4];
  const int m = ghost_images(gx, gy, A, dx, dy, rx, ry);
  lux = lux0;
  luy = luy0;
  lphi = 0.0;
  for (int j = 0; j < m; ++j) {
    const int qx = px + dx[j] + 3, qy = py + dy[j] + 3;
    const double lqx = L.lq[0][qy][qx], lqy = L.lq[1][qy][qx];
    const double sg = ((rx[j] + ry[j]) & 1) ? -1.0 : 1.0;
    lux += sg * phi * lqx;
    luy += sg * phi * lqy;
    double uex = ux, uey = uy;   // the ghost velocity of this image (x first, then y)
    if (rx[j]) {
      const double w = (gx + dx[j]) < 0 ? A.c.uw_lo : A.c.uw_hi;
      uex = -uex;
      uey = 2.0 * w - uey;
    }
    if (ry[j]) {
      const double w = (gy + dy[j]) < 0 ? A.c.uw_lo : A.c.uw_hi;
      uex = 2.0 * w - uex;
      uey = -uey;
    }
    lphi += uex * lqx + uey * lqy;
  }
}

template <int FORM, int BC>
__global__ __launch_bounds__(kAT) void k_adj_b(AArgs A) {
  __shared__ AdjLds L;
  constexpr bool WX = (BC & 1) != 0, WY = (BC & 2) != 0;
  const int ntx = (A.nx + AS::TX - 1) / AS::TX, nty = (A.ny + AS::TY - 1) / AS::TY;
  int tile_x, tile_y;
  if (!xcd_tile(ntx, nty, tile_x, tile_y)) return;
  const StepArgs& a = A.a;
  const ACon& C = A.c;
  const int tid = threadIdx.x;
  const int N = A.nx * A.ny;
  const int x0 = tile_x * AS::TX, y0 = tile_y * AS::TY;
  const double* sc = A.scr;
  const double kap = C.kappa;

  // phase 0: phi (halo 4) and the adjoint of D (halo 3)
  for (int k = tid; k < kH4H * kH4W; k += kAT) {
    const int py = k / kH4W, px = k - py * kH4W;
    int r;
    const int gx = ext_map(x0 + px - 4, A.nx, WX, r), gy = ext_map(y0 + py - 4, A.ny, WY, r);
    L.phi[py][px] = a.phi[(unsigned)(gy * a.g.pitch + gx)];
  }
  for (int k = tid; k < kH3H * kH3W; k += kAT) {
    const int py = k / kH3W, px = k - py * kH3W;
    int n;
    L.ld[py][px] = window_node(x0 + px - 3, y0 + py - 3, A, n) ? sc[(size_t)kSD * N + n] : 0.0;
  }
  __syncthreads();

  // phase 1: grad and lap of phi (Eqs. 41-42) on halo 3; the adjoint of the
  // node field phi u from D(x) = 3 sum_i w_i c_i . (phi u)(x + c_i), gathered
  // from the nodes that read each position (halo 3; zero beyond the window)
  for (int k = tid; k < kH3H * kH3W; k += kAT) {
    const int py = k / kH3W, px = k - py * kH3W;
    const double pc = L.phi[py + 1][px + 1];
    double gx = 0.0, gy = 0.0, l = 0.0, qx = 0.0, qy = 0.0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const double v = L.phi[py + 1 + cy(i)][px + 1 + cx(i)];
      gx += wtd(i) * cx(i) * v;
      gy += wtd(i) * cy(i) * v;
      l += wtd(i) * (v - pc);
      const int sy = py - cy(i), sx = px - cx(i);
      const double d = (sy >= 0 && sy < kH3H && sx >= 0 && sx < kH3W) ? L.ld[sy][sx] : 0.0;
      qx += 3.0 * wtd(i) * cx(i) * d;
      qy += 3.0 * wtd(i) * cy(i) * d;
    }
    L.gl[0][py][px] = 3.0 * gx;
    L.gl[1][py][px] = 3.0 * gy;
    L.gl[2][py][px] = 6.0 * l;
    L.lq[0][py][px] = qx;
    L.lq[1][py][px] = qy;
  }
  __syncthreads();

  // phase 2: at every node of halo 2, the adjoint of F_sf: u = (j + cs^2 F/2)/(cs^2 rho)
  // gives lambda_F += lambda_u / (2 rho) with lambda_u complete (its div part
  // included); CSF also the adjoint of div n at the node
  for (int k = tid; k < kH2H * kH2W; k += kAT) {
    const int py = k / kH2W, px = k - py * kH2W;
    const int gxn = x0 + px - 2, gyn = y0 + py - 2;
    int n;
    double lfx = 0.0, lfy = 0.0, ldn = 0.0;
    if (window_node(gxn, gyn, A, n)) {
      const double phi = L.phi[py + 2][px + 2];
      const double rho = C.rho2 + C.drho_h * (1.0 + phi);
      double lux, luy, lph;
      u_adjoint(L, A, px - 2, py - 2, gxn, gyn, sc[(size_t)kSVX * N + n], sc[(size_t)kSVY * N + n], phi,
                sc[(size_t)kSUX * N + n], sc[(size_t)kSUY * N + n], lux, luy, lph);
      lfx = sc[(size_t)kSFX * N + n] + 0.5 * lux / rho;
      lfy = sc[(size_t)kSFY * N + n] + 0.5 * luy / rho;
      if constexpr (FORM >= 6) {   // the adjoint of div n at the node; n = G / sqrt(|G|^2 + eps^2)  (A8)
        const int qy = py + 1, qx = px + 1;   // halo-3 index of this node
        const double gx = L.gl[0][qy][qx], gy = L.gl[1][qy][qx];
        if constexpr (FORM == 6) {   // F = -kappa |G|^2 n div n
          const double inv = 1.0 / sqrt(gx * gx + gy * gy + C.eps2);
          ldn = -kap * (gx * gx + gy * gy) * (gx * inv * lfx + gy * inv * lfy);
        } else {                     // F = -(sigma/2) G div n
          ldn = -0.5 * C.sigma * (gx * lfx + gy * lfy);
        }
      }
    }
    L.lf[0][py][px] = lfx;
    L.lf[1][py][px] = lfy;
    L.lf[2][py][px] = ldn;
  }
  __syncthreads();

  // phase 3: at every position of halo 1 (nodes, and ghost positions one
  // step beyond a wall), the adjoints of grad phi, lap phi and mu_phi: from
  // the force form's stencils (gathered from the nodes whose force reads the
  // position), from grad rho and h^eq at nodes, then mu_phi = 4 beta phi
  // (phi^2 - 1) - kappa lap phi  (Eq. 2).  dL/dsigma: the terms of mu_phi
  // (which is proportional to sigma) at the positions this tile owns.
  double gsig = 0.0;
  for (int k = tid; k < kH1H * kH1W; k += kAT) {
    const int py = k / kH1W, px = k - py * kH1W;
    const int gxn = x0 + px - 1, gyn = y0 + py - 1;
    const int qy = py + 2, qx = px + 2;          // halo-3 index
    const int ry = py + 1, rx = px + 1;          // halo-2 index
    const double phi = L.phi[py + 3][px + 3];
    const double gx = L.gl[0][qy][qx], gy = L.gl[1][qy][qx], lp = L.gl[2][qy][qx];
    int n;
    const bool node = window_node(gxn, gyn, A, n);
    double lgx = 0.0, lgy = 0.0, ll = 0.0, lmu = 0.0;
    if (node) {
      lgx += C.drho_h * sc[(size_t)kSGX * N + n];   // grad rho = (rho1 - rho2)/2 grad phi
      lgy += C.drho_h * sc[(size_t)kSGY * N + n];
      lmu += sc[(size_t)kSMU * N + n];               // h^eq (Eq. 32)
    }
    if constexpr (FORM == 0 || FORM == 1) {
      // F(x) = 3 sum_i w_i [c_ix T_xx + c_iy T_xy ; c_ix T_xy + c_iy T_yy](x + c_i)
      double ltxx = 0.0, ltxy = 0.0, ltyy = 0.0;
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const double ax = L.lf[0][ry - cy(i)][rx - cx(i)], ay = L.lf[1][ry - cy(i)][rx - cx(i)];
        const double w = 3.0 * wtd(i);
        ltxx += w * cx(i) * ax;
        ltxy += w * (cy(i) * ax + cx(i) * ay);
        ltyy += w * cy(i) * ay;
      }
      if constexpr (FORM == 0) {   // T = -kappa G (x) G
        lgx += -kap * (2.0 * gx * ltxx + gy * ltxy);
        lgy += -kap * (gx * ltxy + 2.0 * gy * ltyy);
      } else {                     // T = kappa (|G|^2 I - G (x) G)
        lgx += kap * (-gy * ltxy + 2.0 * gx * ltyy);
        lgy += kap * (2.0 * gy * ltxx - gx * ltxy);
      }
    } else if constexpr (FORM == 2 || FORM == 5) {
      // CPF-1: F = -phi grad mu;  PF-2: F = kappa phi grad lap phi
      double acc = 0.0;
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const double ax = L.lf[0][ry - cy(i)][rx - cx(i)], ay = L.lf[1][ry - cy(i)][rx - cx(i)];
        acc += 3.0 * wtd(i) * (cx(i) * ax + cy(i) * ay) * L.phi[py + 3 - cy(i)][px + 3 - cx(i)];
      }
      if constexpr (FORM == 2) lmu += -acc;
      else ll += kap * acc;
    } else if constexpr (FORM == 3) {   // CPF-2: F = mu G
      if (node) {
        const double lfx = L.lf[0][ry][rx], lfy = L.lf[1][ry][rx];
        const double mu = C.beta4 * phi * (phi * phi - 1.0) - kap * lp;
        lmu += gx * lfx + gy * lfy;
        lgx += mu * lfx;
        lgy += mu * lfy;
      }
    } else if constexpr (FORM == 4) {   // PF-1: F = -kappa G lap phi
      if (node) {
        const double lfx = L.lf[0][ry][rx], lfy = L.lf[1][ry][rx];
        lgx += -kap * lp * lfx;
        lgy += -kap * lp * lfy;
        ll += -kap * (gx * lfx + gy * lfy);
      }
    } else {   // CSF: div n gathers, the node-local terms, then n(G)
      double lnx = 0.0, lny = 0.0;
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const double d = 3.0 * wtd(i) * L.lf[2][ry - cy(i)][rx - cx(i)];
        lnx += cx(i) * d;
        lny += cy(i) * d;
      }
      const double s = sqrt(gx * gx + gy * gy + C.eps2);
      if (node) {
        const double lfx = L.lf[0][ry][rx], lfy = L.lf[1][ry][rx];
        double dn = 0.0;
#pragma unroll
        for (int i = 1; i < 9; ++i) {
          const double ax = L.gl[0][qy + cy(i)][qx + cx(i)], ay = L.gl[1][qy + cy(i)][qx + cx(i)];
          const double inv = 1.0 / sqrt(ax * ax + ay * ay + C.eps2);
          dn += wtd(i) * (cx(i) * ax * inv + cy(i) * ay * inv);
        }
        dn *= 3.0;
        if constexpr (FORM == 6) {
          const double g2 = gx * gx + gy * gy, nx = gx / s, ny = gy / s;
          lnx += -kap * g2 * dn * lfx;
          lny += -kap * g2 * dn * lfy;
          const double t = -kap * 2.0 * dn * (nx * lfx + ny * lfy);
          lgx += t * gx;
          lgy += t * gy;
        } else {
          lgx += -0.5 * C.sigma * dn * lfx;
          lgy += -0.5 * C.sigma * dn * lfy;
        }
      }
      const double gn = (gx * lnx + gy * lny) / (s * s * s);
      lgx += lnx / s - gx * gn;
      lgy += lny / s - gy * gn;
    }
    // mu_phi at this position
    const double mu = C.beta4 * phi * (phi * phi - 1.0) - kap * lp;
    ll += -kap * lmu;
    L.la[0][py][px] = lgx;
    L.la[1][py][px] = lgy;
    L.la[2][py][px] = ll;
    L.la[3][py][px] = C.beta4 * (3.0 * phi * phi - 1.0) * lmu;
    // the tile owns a position whose node (or, beyond a wall, mirror node) is in the tile
    int r;
    const int mx = ext_map(gxn, A.nx, WX, r), my = ext_map(gyn, A.ny, WY, r);
    const bool own = (WX || (gxn >= 0 && gxn < A.nx)) && (WY || (gyn >= 0 && gyn < A.ny)) && mx >= x0 &&
                     mx < x0 + AS::TX && my >= y0 && my < y0 + AS::TY && mx < A.nx && my < A.ny;
    if (own) gsig += lmu * mu / C.sigma;
  }
  __syncthreads();

  // phase 4: the adjoint of the extended phi on halo 2 from the transposed
  // stencils: G(z) = 3 sum_i w_i c_i phi(z + c_i), L(z) = 6 sum_i w_i (phi(z + c_i) - phi(z))
  for (int k = tid; k < kH2H * kH2W; k += kAT) {
    const int py = k / kH2W, px = k - py * kH2W;
    const int ay = py - 1, ax = px - 1;   // halo-1 index of this position (may be outside)
    const bool in1 = ay >= 0 && ay < kH1H && ax >= 0 && ax < kH1W;
    double acc = in1 ? L.la[3][ay][ax] - 6.0 * (1.0 - wtd(0)) * L.la[2][ay][ax] : 0.0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const int sy = ay - cy(i), sx = ax - cx(i);
      if (sy >= 0 && sy < kH1H && sx >= 0 && sx < kH1W)
        acc += 3.0 * wtd(i) * (cx(i) * L.la[0][sy][sx] + cy(i) * L.la[1][sy][sx]) + 6.0 * wtd(i) * L.la[2][sy][sx];
    }
    L.lp[py][px] = acc;
  }
  __syncthreads();

  // phase 5: lambda_n of the tile's nodes
  const int lx = tid & (AS::TX - 1), ty = tid / AS::TX;
  const int x = x0 + lx, y = y0 + ty;
  if (x < A.nx && y < A.ny) {
    const int k = y * A.nx + x;
    const double phi = L.phi[ty + 4][lx + 4];
    const double rho = C.rho2 + C.drho_h * (1.0 + phi);
    const double muv = C.mu2 + C.dmu_h * (1.0 + phi);
    const double ux = sc[(size_t)kSVX * N + k], uy = sc[(size_t)kSVY * N + k];
    double lux, luy, lph;
    u_adjoint(L, A, lx, ty, x, y, ux, uy, phi, sc[(size_t)kSUX * N + k], sc[(size_t)kSUY * N + k], lux, luy, lph);
    const double lfx = L.lf[0][ty + 2][lx + 2], lfy = L.lf[1][ty + 2][lx + 2];   // adjoint of F
    double lrho = sc[(size_t)kSRHO * N + k] - (ux * lux + uy * luy) / rho + C.gx * lfx + C.gy * lfy;
    double lphi = sc[(size_t)kSPHI * N + k] + lph + C.drho_h * lrho;
    if constexpr (FORM == 2 || FORM == 5) {   // point-wise phi factor of CPF-1 / PF-2
      const int qy = ty + 3, qx = lx + 3;
      double ax = 0.0, ay = 0.0;
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const double lpp = L.gl[2][qy + cy(i)][qx + cx(i)];
        const double pp = L.phi[qy + 1 + cy(i)][qx + 1 + cx(i)];
        const double v = FORM == 2 ? C.beta4 * pp * (pp * pp - 1.0) - kap * lpp : lpp;
        ax += wtd(i) * cx(i) * v;
        ay += wtd(i) * cy(i) * v;
      }
      const double s = FORM == 2 ? -3.0 : 3.0 * kap;
      lphi += s * (ax * lfx + ay * lfy);
    }
    // sigma enters F_sf linearly except through mu_phi (CPF forms)
    if constexpr (FORM != 2 && FORM != 3)
      gsig += (sc[(size_t)kSFSX * N + k] * lfx + sc[(size_t)kSFSY * N + k] * lfy) / C.sigma;
    // fold the phi adjoint of this node's images within two steps beyond a wall
    {
      int ppx[3], prx[3], ppy[3], pry[3];
      const int mx = WX ? preimages(x, A.nx, 1, 2, ppx, prx) : 1;
      const int my = WY ? preimages(y, A.ny, 1, 2, ppy, pry) : 1;
      if (!WX) ppx[0] = x;
      if (!WY) ppy[0] = y;
      for (int i = 0; i < mx; ++i)
        for (int j = 0; j < my; ++j) lphi += L.lp[ppy[j] - y0 + 2][ppx[i] - x0 + 2];
    }
    const double tauf = 0.5 + muv / (kC2 * rho);
    const double om = 1.0 / tauf, omh = C.inv_tau_h;
    const double ljx = lux / (kC2 * rho), ljy = luy / (kC2 * rho);
    const double lS = sc[(size_t)kSP * N + k];
    double lfp[9], lhp[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      int tx = x + cx(i), tyy = y + cy(i);
      bool h = false;
      if (tx < 0 || tx >= A.nx) { if (WX) h = true; else tx = tx < 0 ? tx + A.nx : tx - A.nx; }
      if (tyy < 0 || tyy >= A.ny) { if (WY) h = true; else tyy = tyy < 0 ? tyy + A.ny : tyy - A.ny; }
      const int slot = h ? opp(i) : i;
      const int tgt = h ? k : tyy * A.nx + tx;
      lfp[i] = A.lin[(size_t)slot * N + tgt];
      lhp[i] = A.lin[(size_t)(9 + slot) * N + tgt];
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      A.lout[(size_t)i * N + k] = (1.0 - om) * lfp[i] + (cx(i) * ljx + cy(i) * ljy) + lS;
      A.lout[(size_t)(9 + i) * N + k] = (1.0 - omh) * lhp[i] + lphi;
    }
  }
  const double tot = block_sum(gsig, L.red);
  if (tid == 0) A.gsig[tile_y * ntx + tile_x] += tot;
}

// ---------------------------------------------------------------------------
// Adjoint of the initial state (reading A11): f = f^eq(0, rho(phi0), u0),
// h = h^eq(phi0, mu(phi0), u0), J = phi0 u0.
// ---------------------------------------------------------------------------
struct IBuf {
  double *phie2;           // phi0 extended by two layers
  double *lphi, *lmun;     // interior: adjoint of phi0 (point-wise part), of mu0 via h^eq
  double *lL1, *lphie1;    // e1: adjoint of lap phi0 and the point-wise phi part of mu0
  double *gsig, *gM;       // e1: dL/dsigma and dL/dM terms of the initial state
};

__global__ __launch_bounds__(kB) void k_adj_fa_init(AGrid g, const float* __restrict__ phi0, double* __restrict__ phie2) {
  const int ne = (g.nx + 4) * (g.ny + 4);
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= ne) return;
  const int ex = k % (g.nx + 4) - 2, ey = k / (g.nx + 4) - 2;
  int r;
  const int x = ext_map(ex, g.nx, g.wx, r), y = ext_map(ey, g.ny, g.wy, r);
  phie2[k] = (double)phi0[i0(g, x, y)];
}

// Step 1: node-local part.
__global__ __launch_bounds__(kB) void k_adj_init_a(AGrid g, ACon c, IBuf b, const float* __restrict__ phi0,
                                                   const float* __restrict__ ux0, const float* __restrict__ uy0,
                                                   const double* __restrict__ lam) {
  const int N = g.nx * g.ny;
  const int n = blockIdx.x * kB + threadIdx.x;
  if (n >= N) return;
  const double ux = ux0 ? ux0[n] : 0.0, uy = uy0 ? uy0[n] : 0.0;
  const double usq = ux * ux + uy * uy;
  double lrho = 0, lphi = 0, lmu = 0;
  for (int i = 0; i < 9; ++i) {
    const double cu = cx(i) * ux + cy(i) * uy;
    const double si = 3.0 * cu + 4.5 * cu * cu - 1.5 * usq;
    lrho += wtd(i) * kC2 * si * lam[(size_t)i * N + n];
    const double lh = lam[(size_t)(9 + i) * N + n];
    if (i == 0) { lphi += lh; lmu += (wtd(0) - 1.0) * lh; }
    else { lphi += 3.0 * wtd(i) * cu * lh; lmu += wtd(i) * lh; }
  }
  lphi += ux * lam[(size_t)18 * N + n] + uy * lam[(size_t)19 * N + n];
  lphi += c.drho_h * lrho;
  b.lphi[n] = lphi;
  b.lmun[n] = lmu;   // sum_i wbar'_i lambda_h_i (h^eq depends on eta mu)
}

// Step 2 (e1 grid): mu0 = 4 beta phi (phi^2 - 1) - kappa lap(phi0)
__global__ __launch_bounds__(kB) void k_adj_init_b(AGrid g, ACon c, IBuf b) {
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
  b.gsig[k] = in ? lmu * mu / c.sigma : 0.0;
  b.gM[k] = in ? sw * mu * c.detadM : 0.0;
  b.lL1[k] = in ? -c.kappa * lmu : 0.0;
  b.lphie1[k] = in ? c.beta4 * (3.0 * p * p - 1.0) * lmu : 0.0;
}

// Step 3: transposed Laplacian onto e1 positions, folded onto the nodes.
__global__ __launch_bounds__(kB) void k_adj_init_c(AGrid g, IBuf b, double* __restrict__ dphi0) {
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

// Deterministic two-level sum: one partial sum per block (grid-stride over
// gridDim.x blocks), then one block sums the partials.
__global__ __launch_bounds__(kB) void k_sum_part(const double* __restrict__ a, long long n, double* __restrict__ part) {
  __shared__ double red[kB];
  double s = 0.0;
  for (long long k = (long long)blockIdx.x * kB + threadIdx.x; k < n; k += (long long)gridDim.x * kB) s += a[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kB) void k_sum_fin(const double* __restrict__ part, int npart, double* out) {
  __shared__ double red[kB];
  double s = 0.0;
  for (int k = threadIdx.x; k < npart; k += kB) s += part[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// lambda_T of L = 1/2 sum (phi_T - phi*)^2 (reading A19): dL/dh_i = phi_T - phi*.
__global__ __launch_bounds__(kB) void k_adj_seed(AGrid g, const double* __restrict__ phi, int pitch,
                                                 const float* __restrict__ target, double* __restrict__ lam,
                                                 double* __restrict__ lossd) {
  const int N = g.nx * g.ny;
  const int k = blockIdx.x * kB + threadIdx.x;
  if (k >= N) return;
  const int x = k % g.nx, y = k / g.nx;
  const double r = phi[(long long)y * pitch + x] - (double)target[k];
  for (int i = 0; i < 9; ++i) {
    lam[(size_t)i * N + k] = 0.0;
    lam[(size_t)(9 + i) * N + k] = r;   // phi = sum_i h_i
  }
  lam[(size_t)18 * N + k] = 0.0;
  lam[(size_t)19 * N + k] = 0.0;
  lossd[k] = 0.5 * r * r;
}

unsigned nblk(long long n) { return (unsigned)((n + kB - 1) / kB); }

template <int FORM, int BC>
void launch_adj_t(const AArgs& A, dim3 grid, hipStream_t st) {
  hipLaunchKernelGGL((k_adj_a<FORM, BC>), grid, dim3(kAT), 0, st, A);
  hipLaunchKernelGGL((k_adj_b<FORM, BC>), grid, dim3(kAT), 0, st, A);
}

template <int FORM>
void launch_adj_form(const AArgs& A, dim3 grid, hipStream_t st) {
  switch (A.wx | (A.wy << 1)) {
    case 0: launch_adj_t<FORM, 0>(A, grid, st); break;
    case 1: launch_adj_t<FORM, 1>(A, grid, st); break;
    case 2: launch_adj_t<FORM, 2>(A, grid, st); break;
    default: launch_adj_t<FORM, 3>(A, grid, st); break;
  }
}

hipError_t launch_adjoint(int form, const AArgs& A, hipStream_t st) {
  const int ntiles = ((A.nx + AS::TX - 1) / AS::TX) * ((A.ny + AS::TY - 1) / AS::TY);
  const dim3 grid((ntiles + kXcds - 1) / kXcds * kXcds);
  switch (form) {
    case 0: launch_adj_form<0>(A, grid, st); break;
    case 1: launch_adj_form<1>(A, grid, st); break;
    case 2: launch_adj_form<2>(A, grid, st); break;
    case 3: launch_adj_form<3>(A, grid, st); break;
    case 4: launch_adj_form<4>(A, grid, st); break;
    case 5: launch_adj_form<5>(A, grid, st); break;
    case 6: launch_adj_form<6>(A, grid, st); break;
    default: launch_adj_form<7>(A, grid, st); break;
  }
  return hipGetLastError();
}

}  // namespace

}  // namespace pflbm

// Scratch of lbm_adjoint_step_blob_noalloc: the kNS FP64 planes that k_adj_a
// writes and k_adj_b reads, for lattices of at most kNoallocNodes nodes.  One
// copy lives on every GPU the library runs on, for the life of the process.
// Host code reaches it only through the address hipGetSymbolAddress returns
// on that device (noalloc_scratch below).
constexpr size_t kNoallocBytes = size_t(64) << 20;   // 64 MiB
constexpr long long kNoallocNodes = (long long)(kNoallocBytes / (pflbm::kNS * sizeof(double)));
static __device__ __align__(256) double scratch[kNoallocBytes / sizeof(double)];

using namespace pflbm;

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct lbm_adj {
  lbm_sim* sim;
  lbm_params p;
  AGrid g;
  ACon c;
  Grid sg;         // layout of the simulation's state arrays
  Phys ph;
  int ntiles;
  double* scr;     // kNS planes (the scratch of one adjoint step)
  double* gsig;    // per-tile accumulators
  double* gM;
  IBuf ib;         // adjoint of the initial state
  double* lossd;   // per-node loss terms
  double* part;    // kRed partial sums
  double* red;     // 4 results
};

namespace {

size_t adj_tiles(const lbm_params* p) {
  return (size_t)((p->nx + AS::TX - 1) / AS::TX) * (size_t)((p->ny + AS::TY - 1) / AS::TY);
}

// Doubles of the adjoint workspace, in the order lbm_adjoint_create carves it.
size_t adj_doubles(const lbm_params* p) {
  const size_t N = (size_t)p->nx * p->ny, N1 = (size_t)(p->nx + 2) * (p->ny + 2),
               N2 = (size_t)(p->nx + 4) * (p->ny + 4);
  const size_t T = adj_tiles(p);
  // scratch, tile accumulators, init (phie2, lphi, lmun, lL1, lphie1, gsig, gM), loss terms, partials, results
  return (size_t)kNS * N + 2 * T + N2 + 2 * N + 4 * N1 + N + kRed + 8;
}

int adj_sum(const double* a, long long n, double* part, double* out, hipStream_t st) {
  const long long nb = (n + kB - 1) / kB;
  const int np = nb < 1 ? 1 : (nb < kRed ? (int)nb : kRed);   // at most kRed partial sums
  hipLaunchKernelGGL(k_sum_part, dim3(np), dim3(kB), 0, st, a, n, part);
  hipLaunchKernelGGL(k_sum_fin, dim3(1), dim3(kB), 0, st, part, np, out);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LBM_OK : set_error(LBM_E_HIP, "adjoint sum: %s", hipGetErrorString(e));
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
  if (p.wall_x == 2 || p.wall_y == 2)
    return set_error(LBM_E_UNSUPPORTED, "the adjoint supports periodic and no-slip walls only");
  lbm_adj* a = new (std::nothrow) lbm_adj();
  if (!a) return set_error(LBM_E_INVAL, "out of host memory");
  a->sim = sim;
  a->p = p;
  const int nx = p.nx, ny = p.ny;
  a->g.nx = nx; a->g.ny = ny; a->g.wx = p.wall_x; a->g.wy = p.wall_y;
  {
    SimView v;
    if (int r = sim_view(sim, &v)) { delete a; return r; }
    a->sg = v.g;
  }
  a->ph = sim_phys(sim);
  const Phys& ph = a->ph;
  ACon& c = a->c;
  c.beta4 = ph.beta4_d; c.kappa = ph.kappa_d; c.sigma = p.sigma; c.eps2 = ph.eps2_d;
  c.eta = ph.eta_d; c.detadM = 1.0 / (kC2 * (p.tau_h - 0.5)); c.a_h = ph.a_h_d; c.inv_tau_h = ph.inv_tau_h_d;
  c.rho2 = ph.rho2_d; c.drho_h = ph.drho_half_d; c.mu2 = ph.mu2_d; c.dmu_h = ph.dmu_half_d;
  c.gx = ph.gx_d; c.gy = ph.gy_d; c.rho0 = ph.rho0_d; c.uw_lo = ph.uw_lo_d; c.uw_hi = ph.uw_hi_d;
  const size_t N = (size_t)nx * ny, N1 = (size_t)(nx + 2) * (ny + 2), N2 = (size_t)(nx + 4) * (ny + 4);
  a->ntiles = (int)adj_tiles(&p);
  double* q = (double*)d_ws;
  auto take = [&](size_t n) { double* r = q; q += n; return r; };
  a->scr = take((size_t)kNS * N);
  a->gsig = take((size_t)a->ntiles);
  a->gM = take((size_t)a->ntiles);
  a->ib.phie2 = take(N2);
  a->ib.lphi = take(N);
  a->ib.lmun = take(N);
  a->ib.lL1 = take(N1);
  a->ib.lphie1 = take(N1);
  a->ib.gsig = take(N1);
  a->ib.gM = take(N1);
  a->lossd = take(N);
  a->part = take(kRed);
  a->red = take(8);
  *out = a;
  return lbm_adjoint_reset(a, nullptr);
}

int lbm_adjoint_reset(lbm_adj* a, void* stream) {
  if (!a) return set_error(LBM_E_INVAL, "adjoint is NULL");
  const long long N1 = (long long)(a->p.nx + 2) * (a->p.ny + 2);
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_adj_zero, dim3(nblk(2LL * a->ntiles)), dim3(kB), 0, st, a->gsig, 2LL * a->ntiles);
  hipLaunchKernelGGL(k_adj_zero, dim3(nblk(2 * N1)), dim3(kB), 0, st, a->ib.gsig, 2 * N1);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LBM_OK : set_error(LBM_E_HIP, "adjoint reset: %s", hipGetErrorString(e));
}

int lbm_adjoint_seed_phi_misfit(lbm_adj* a, const float* d_target, double* d_lambda, double* h_loss, void* stream) {
  if (!a || !d_target || !d_lambda) return set_error(LBM_E_INVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  const long long N = (long long)a->p.nx * a->p.ny;
  SimView v;
  if (int r = sim_view(a->sim, &v)) return r;
  hipLaunchKernelGGL(k_adj_seed, dim3(nblk(N)), dim3(kB), 0, st, a->g, v.phi, v.g.pitch, d_target, d_lambda, a->lossd);
  if (int r = adj_sum(a->lossd, N, a->part, a->red + 2, st)) return r;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && h_loss) {
    e = hipMemcpyAsync(h_loss, a->red + 2, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  return e == hipSuccess ? LBM_OK : set_error(LBM_E_HIP, "adjoint seed: %s", hipGetErrorString(e));
}

namespace {

int adjoint_step_at(lbm_adj* a, const float* S, const double* phis, int32_t form, const double* lin, double* lout,
                    double* scr, hipStream_t st) {
  if (form < 0 || form >= LBM_NUM_FORMS) return set_error(LBM_E_INVAL, "bad force form %d", form);
  const size_t N = (size_t)a->p.nx * a->p.ny;
  if (!lin || !lout) return set_error(LBM_E_INVAL, "NULL argument");
  const char *ib = (const char*)lin, *ob = (const char*)lout;
  if (ib < ob + 20 * N * sizeof(double) && ob < ib + 20 * N * sizeof(double))
    return set_error(LBM_E_INVAL, "lambda_in and lambda_out must not overlap");
  AArgs A{};
  A.a.sin = S;
  A.a.sout = nullptr;
  A.a.phi = phis;
  A.a.status = nullptr;
  A.a.g = a->sg;
  A.a.g.fast = 0;
  A.a.c = a->ph;
  A.lin = lin;
  A.lout = lout;
  A.scr = scr;
  A.gsig = a->gsig;
  A.gM = a->gM;
  A.c = a->c;
  A.nx = a->p.nx;
  A.ny = a->p.ny;
  A.wx = a->p.wall_x != 0;
  A.wy = a->p.wall_y != 0;
  const hipError_t e = launch_adjoint(form, A, st);
  return e == hipSuccess ? LBM_OK : set_error(LBM_E_HIP, "adjoint step: %s", hipGetErrorString(e));
}

}  // namespace

int lbm_adjoint_step(lbm_adj* a, int32_t form, const double* d_lambda_in, double* d_lambda_out, void* stream) {
  if (!a) return set_error(LBM_E_INVAL, "NULL argument");
  SimView v;
  if (int r = sim_view(a->sim, &v)) return r;
  return adjoint_step_at(a, v.s, v.phi, form, d_lambda_in, d_lambda_out, a->scr, (hipStream_t)stream);
}

int lbm_adjoint_step_blob(lbm_adj* a, const void* d_blob, int32_t form, const double* d_lambda_in,
                          double* d_lambda_out, void* stream) {
  if (!a || !d_blob) return set_error(LBM_E_INVAL, "NULL argument");
  const char* b = (const char*)d_blob;   // lbm_save layout: state array, then phi
  const size_t sb = (size_t)kNPL * (size_t)a->sg.ps * sizeof(float);
  return adjoint_step_at(a, (const float*)b, (const double*)(b + sb), form, d_lambda_in, d_lambda_out, a->scr,
                         (hipStream_t)stream);
}

}  // extern "C"

namespace {

// Device address of `scratch` on the current device, looked up once per device.
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

int noalloc_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(LBM_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(LBM_E_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(LBM_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_noalloc_ptr[dev] = p;
  }
  *out = (double*)g_noalloc_ptr[dev];
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_adjoint_step_blob_noalloc(lbm_adj* a, const void* d_blob, int32_t form, const double* d_lambda_in,
                                  double* d_lambda_out, void* stream) {
  if (!a || !d_blob) return set_error(LBM_E_INVAL, "NULL argument");
  const long long n = (long long)a->p.nx * a->p.ny;
  if (n > kNoallocNodes)
    return set_error(LBM_E_INVAL, "lattice of %lld nodes: lbm_adjoint_step_blob_noalloc takes at most %lld", n,
                     kNoallocNodes);
  double* scr = nullptr;
  if (int r = noalloc_scratch(&scr)) return r;
  const char* b = (const char*)d_blob;
  const size_t sb = (size_t)kNPL * (size_t)a->sg.ps * sizeof(float);
  return adjoint_step_at(a, (const float*)b, (const double*)(b + sb), form, d_lambda_in, d_lambda_out, scr,
                         (hipStream_t)stream);
}

int lbm_adjoint_init(lbm_adj* a, const float* d_phi0, const float* d_ux0, const float* d_uy0, const double* d_lambda0,
                     double* d_dphi0, void* stream) {
  if (!a || !d_phi0 || !d_lambda0 || !d_dphi0) return set_error(LBM_E_INVAL, "NULL argument");
  if ((d_ux0 == nullptr) != (d_uy0 == nullptr)) return set_error(LBM_E_INVAL, "give both u0 components or neither");
  hipStream_t st = (hipStream_t)stream;
  const AGrid& g = a->g;
  const long long N = (long long)g.nx * g.ny, N1 = (long long)(g.nx + 2) * (g.ny + 2);
  hipLaunchKernelGGL(k_adj_fa_init, dim3(nblk((long long)(g.nx + 4) * (g.ny + 4))), dim3(kB), 0, st, g, d_phi0,
                     a->ib.phie2);
  hipLaunchKernelGGL(k_adj_init_a, dim3(nblk(N)), dim3(kB), 0, st, g, a->c, a->ib, d_phi0, d_ux0, d_uy0, d_lambda0);
  hipLaunchKernelGGL(k_adj_init_b, dim3(nblk(N1)), dim3(kB), 0, st, g, a->c, a->ib);
  hipLaunchKernelGGL(k_adj_init_c, dim3(nblk(N)), dim3(kB), 0, st, g, a->ib, d_dphi0);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LBM_OK : set_error(LBM_E_HIP, "adjoint init: %s", hipGetErrorString(e));
}

int lbm_adjoint_param_grads(lbm_adj* a, double* h_dsigma, double* h_dM, void* stream) {
  if (!a || !h_dsigma || !h_dM) return set_error(LBM_E_INVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  const long long N1 = (long long)(a->p.nx + 2) * (a->p.ny + 2);
  if (int r = adj_sum(a->gsig, a->ntiles, a->part, a->red + 4, st)) return r;
  if (int r = adj_sum(a->gM, a->ntiles, a->part, a->red + 5, st)) return r;
  if (int r = adj_sum(a->ib.gsig, N1, a->part, a->red + 6, st)) return r;
  if (int r = adj_sum(a->ib.gM, N1, a->part, a->red + 7, st)) return r;
  double h[4];
  hipError_t e = hipMemcpyAsync(h, a->red + 4, 4 * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return set_error(LBM_E_HIP, "adjoint grads: %s", hipGetErrorString(e));
  *h_dsigma = h[0] + h[2];
  *h_dM = h[1] + h[3];
  return LBM_OK;
}

int lbm_adjoint_destroy(lbm_adj* a) {
  delete a;
  return LBM_OK;
}

}  // extern "C"
