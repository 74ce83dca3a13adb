// Tile machinery shared by the step kernels (lbm_kernels.hip) and the
// adjoint kernels (lbm_adjoint.hip): tile shapes, the LDS layout of a tile,
// the isotropic stencils (Eqs. 41-42), the chemical potential (Eq. 2), the
// eight interfacial forces (Sec. II.B), the pulled populations of a node
// (Eqs. 29-30 in pull form, Eq. 43 pre-applied) and the moments (Eq. 37).
// Everything lives in an unnamed namespace: each translation unit that
// includes this header gets its own copy of these inline device functions.
#pragma once

#include "lbm_internal.hpp"

namespace pflbm {

namespace {

constexpr float CS2 = 1.0f / 3.0f;
constexpr int kXcds = 8;                    // accelerator complex dies of the MI355X

// Tile shape of the fused and order-parameter kernels: TX x TY nodes, one
// per thread.  TX is 32 or 64 (a wavefront covers one or two tile rows, each
// a run inside one 64-node row segment of the state arrays).
template <int TX_, int TY_>
struct Shape {
  static constexpr int TX = TX_, TY = TY_, NT = TX_ * TY_;
  static constexpr int PW = TX + 6, PH = TY + 6;   // phi tile (halo 3)
  static constexpr int BW = TX + 4, BH = TY + 4;   // second-level fields (halo 2)
  static constexpr int UW = TX + 2, UH = TY + 2;   // velocity ring (halo 1)
  static constexpr int NRING = 2 * UW + 2 * TY;    // positions of the velocity ring
  static constexpr int NPHI = (PW * PH + NT - 1) / NT;   // phi values a thread stages
  static_assert(TX == 32 || TX == 64, "a tile row is half or all of a 64-node row segment");
  static_assert(NRING <= NT && NPHI <= 3, "one ring position and at most three phi values per thread");
};

__device__ __forceinline__ int wrap_or_reflect(int c, int n, int wall) {
  if (wall) {
    if (c < 0) c = -1 - c;
    else if (c >= n) c = 2 * n - 1 - c;
    return c < 0 ? 0 : (c >= n ? n - 1 : c);   // positions no active node reads
  }
  c %= n;
  return c < 0 ? c + n : c;
}

// Tile-halo coordinate c in [-3, tile end + 3]: one periodic wrap or one
// mirror about the half-way wall.  Every position an active node reads lies
// within [-3, n + 3] (n >= 8), where one step is exact; the clamp keeps the
// positions of a ragged tile that no active node reads inside the array.
template <bool WALL>
__device__ __forceinline__ int halo_coord(int c, int n) {
  if constexpr (WALL) {
    c = c < 0 ? -1 - c : (c >= n ? 2 * n - 1 - c : c);
    return c < 0 ? 0 : c;
  } else {
    c = c < 0 ? c + n : (c >= n ? c - n : c);
    return c < n ? c : n - 1;
  }
}

// Source of the pulled population I for node (x, y) inside the domain: the
// value that left x - c_I in direction I.  If x - c_I lies beyond a no-slip
// wall, or beyond both walls of a corner, the slot opp(I) of x itself holds
// the bounced population (the wall term is applied when it is stored).  A
// link that crosses only a free-slip wall was reflected specularly: it left
// the node beside x along the wall in the mirrored direction.  Returns the
// element index of plane 0 of the source node in a state array; `slot` is
// the direction to read there.
template <int I>
__device__ __forceinline__ size_t src_base(int x, int y, const Grid& g, int wx, int wy, int& slot) {
  int sx = x - cx(I), sy = y - cy(I);
  bool out_x = false, out_y = false;
  if (cx(I) != 0) {
    if (wx) out_x = (sx < 0) | (sx >= g.nx);
    sx = sx < 0 ? sx + g.nx : (sx >= g.nx ? sx - g.nx : sx);
  }
  if (cy(I) != 0) {
    if (wy) out_y = (sy < 0) | (sy >= g.ny);
    sy = sy < 0 ? sy + g.ny : (sy >= g.ny ? sy - g.ny : sy);
  }
  if (out_x && !out_y && g.slip_x) {
    slot = mirror_x(I);
    return nbase(g, x, sy);
  }
  if (out_y && !out_x && g.slip_y) {
    slot = mirror_y(I);
    return nbase(g, sx, y);
  }
  const bool bounce = out_x || out_y;
  slot = bounce ? opp(I) : I;
  return bounce ? nbase(g, x, y) : nbase(g, sx, sy);
}

// Interior tiles (every pull and every halo position inside the domain)
// address a state array from a uniform tile origin with a 32-bit per-thread
// byte offset; the row shift of a pull and the plane are uniform constants,
// so a load or store is one SGPR-base + VGPR-offset + immediate access with
// no vector address arithmetic.  Values used once (a node's own pulled
// populations and (phi u), every store) go through the non-temporal path;
// the ring's pulls, which the neighbouring tile reads again, do not.
template <class T>
__device__ __forceinline__ const T* at(const T* base, unsigned boff) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff);
}
template <class T>
__device__ __forceinline__ T* at(T* base, unsigned boff) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + boff);
}
__device__ __forceinline__ float ld_nt(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }

// Interior tiles address a state array from an origin at plane 0 of node
// (xo, y0 - 2), xo = the first node of the 64-node row segment holding
// x0 - 2 (the leftmost column any pull of the tile reads).
__device__ __forceinline__ int tile_xo(int x0) { return (x0 - 2) & ~63; }

// Byte offsets, from an interior tile's input origin, of plane 0 of the
// nodes (x0 + xr - 1 + k, y0 + yr), k = 0, 1, 2.  A pull of direction I by
// node (x0 + xr, y0 + yr) reads v3[1 - c_Ix] from the origin moved by -c_Iy
// rows.
__device__ __forceinline__ void node_offsets(const Grid& g, int x0, int xr, int yr, unsigned* v3) {
  const int row = (yr + 2) * g.rowe, s0 = tile_xo(x0) >> 6;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int X = x0 + xr + k - 1;
    v3[k] = 4u * (unsigned)(row + ((X >> 6) - s0) * kSegE + (X & 63));
  }
}

// Population plane P pulled in direction I by the node with offsets v3.
template <int I, int P, bool NT>
__device__ __forceinline__ float pull_tile(const float* tin, int rowe, const unsigned* v3) {
  const float* q = at(tin - (long long)cy(I) * rowe + P * 64, v3[1 - cx(I)]);
  if constexpr (NT) return ld_nt(q);
  else return *q;
}

// 1/x in FP64 from an FP32 seed and two Newton steps (exact to ~1 ulp for
// the positive, normal arguments used here: densities, relaxation times).
__device__ __forceinline__ double rcp64(double x) {
  double r = (double)__builtin_amdgcn_rcpf((float)x);   // ~1 ulp FP32 seed
  r = r * (2.0 - x * r);
  r = r * (2.0 - x * r);
  return r;
}

// Mixture density and viscosity (Eqs. 9-10) from the FP64 order parameter,
// written as rho2 + (rho1 - rho2)(1 + phi)/2 so a light phase keeps its
// relative precision.
__device__ __forceinline__ double rho_of(double phi, const Phys& c) { return c.rho2_d + c.drho_half_d * (1.0 + phi); }
__device__ __forceinline__ double mu_of(double phi, const Phys& c) { return c.mu2_d + c.dmu_half_d * (1.0 + phi); }

template <class S>
struct Lds {
  double phi[S::PH][S::PW];
  double gl[3][S::BH][S::BW];   // grad phi (x, y) and lap phi on the 2-ring
  double b[3][S::BH][S::BW];
  float q[2][S::UH][S::UW];     // phi u on the tile and its 1-node ring
};

// gradient and Laplacian of phi at sPhi position (py, px) (Eqs. 41-42), in
// FP64 from differences to the centre value.
template <class S>
__device__ __forceinline__ void grad_lap_phi(const Lds<S>& s, int py, int px, double& gx, double& gy, double& lap) {
  const double c = s.phi[py][px];
  double sx = 0.0, sy = 0.0, sl = 0.0;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const double d = s.phi[py + cy(i)][px + cx(i)] - c;
    if (cx(i) != 0) sx += (wtd(i) * cx(i)) * d;
    if (cy(i) != 0) sy += (wtd(i) * cy(i)) * d;
    sl += wtd(i) * d;
  }
  gx = 3.0 * sx;
  gy = 3.0 * sy;
  lap = 6.0 * sl;
}

// mu_phi = 4 beta phi (phi^2 - 1) - kappa lap(phi)   (Eq. 2)
__device__ __forceinline__ double chem_pot(double phi, double lap, const Phys& c) {
  return c.beta4_d * phi * ((phi - 1.0) * (phi + 1.0)) - c.kappa_d * lap;
}

// isotropic gradient of an LDS field at (by, bx)  (Eq. 41)
template <int BW>
__device__ __forceinline__ void grad_b(const double (*f)[BW], int by, int bx, double& gx, double& gy) {
  const double c = f[by][bx];
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const double d = f[by + cy(i)][bx + cx(i)] - c;
    if (cx(i) != 0) sx += (wtd(i) * cx(i)) * d;
    if (cy(i) != 0) sy += (wtd(i) * cy(i)) * d;
  }
  gx = 3.0 * sx;
  gy = 3.0 * sy;
}

// Stage B: form-specific node field(s) on the 2-ring (FP64: their stencil
// differences are small against their values).
template <int FORM, class S>
__device__ __forceinline__ void stage_b(Lds<S>& s, int tid, const Phys& c) {
  const double kappa = c.kappa_d;
  for (int k = tid; k < S::BH * S::BW; k += S::NT) {
    const int by = k / S::BW, bx = k - by * S::BW;
    const int py = by + 1, px = bx + 1;
    double gx, gy, lap;
    grad_lap_phi(s, py, px, gx, gy, lap);
    s.gl[0][by][bx] = gx;
    s.gl[1][by][bx] = gy;
    s.gl[2][by][bx] = lap;
    if constexpr (FORM == 3 || FORM == 4) {
      // CPF-2, PF-1: pointwise in G and lap phi
    } else if constexpr (FORM == 0) {          // STF-1: T = -kappa G (x) G, F = div T
      s.b[0][by][bx] = -kappa * gx * gx;
      s.b[1][by][bx] = -kappa * gx * gy;
      s.b[2][by][bx] = -kappa * gy * gy;
    } else if constexpr (FORM == 1) {   // STF-2: T = kappa (|G|^2 I - G (x) G)
      s.b[0][by][bx] = kappa * gy * gy;
      s.b[1][by][bx] = -kappa * gx * gy;
      s.b[2][by][bx] = kappa * gx * gx;
    } else if constexpr (FORM == 2) {   // CPF-1: mu_phi
      s.b[0][by][bx] = chem_pot(s.phi[py][px], lap, c);
    } else if constexpr (FORM == 5) {   // PF-2: lap(phi)
      s.b[0][by][bx] = lap;
    } else {                            // CSF-1/2: n = G / sqrt(|G|^2 + eps^2)
      const double inv = 1.0 / sqrt(gx * gx + gy * gy + c.eps2_d);
      s.b[0][by][bx] = gx * inv;
      s.b[1][by][bx] = gy * inv;
    }
  }
}

// Interfacial force at velocity-ring position (uy_, ux_) (Sec. II.B), in FP64.
// sPhi index of that node is (uy_ + 2, ux_ + 2); stage-B index (uy_ + 1, ux_ + 1).
template <int FORM, class S>
__device__ __forceinline__ void force_sf(const Lds<S>& s, int uy_, int ux_, const Phys& c, double& fxo, double& fyo) {
  const int py = uy_ + 2, px = ux_ + 2, by = uy_ + 1, bx = ux_ + 1;
  const double kappa = c.kappa_d;
  double fx, fy;
  if constexpr (FORM == 0 || FORM == 1) {   // div T
    double sx = 0.0, sy = 0.0;
    const double txx = s.b[0][by][bx], txy = s.b[1][by][bx], tyy = s.b[2][by][bx];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const int ny_ = by + cy(i), nx_ = bx + cx(i);
      const double dxx = s.b[0][ny_][nx_] - txx, dxy = s.b[1][ny_][nx_] - txy, dyy = s.b[2][ny_][nx_] - tyy;
      sx += wtd(i) * ((double)cx(i) * dxx + (double)cy(i) * dxy);
      sy += wtd(i) * ((double)cx(i) * dxy + (double)cy(i) * dyy);
    }
    fx = 3.0 * sx;
    fy = 3.0 * sy;
  } else if constexpr (FORM == 2) {         // CPF-1: -phi grad(mu)
    double gx, gy;
    grad_b(s.b[0], by, bx, gx, gy);
    const double phi = s.phi[py][px];
    fx = -phi * gx;
    fy = -phi * gy;
  } else if constexpr (FORM == 3) {         // CPF-2: mu grad(phi)
    const double gx = s.gl[0][by][bx], gy = s.gl[1][by][bx], lap = s.gl[2][by][bx];
    const double mu = chem_pot(s.phi[py][px], lap, c);
    fx = mu * gx;
    fy = mu * gy;
  } else if constexpr (FORM == 4) {         // PF-1: -kappa grad(phi) lap(phi)
    const double gx = s.gl[0][by][bx], gy = s.gl[1][by][bx], lap = s.gl[2][by][bx];
    fx = -kappa * gx * lap;
    fy = -kappa * gy * lap;
  } else if constexpr (FORM == 5) {         // PF-2: kappa phi grad(lap phi)
    double gx, gy;
    grad_b(s.b[0], by, bx, gx, gy);
    const double k = kappa * s.phi[py][px];
    fx = k * gx;
    fy = k * gy;
  } else {                                  // CSF: div n
    double dn = 0.0;
    const double nxc = s.b[0][by][bx], nyc = s.b[1][by][bx];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const double dx = s.b[0][by + cy(i)][bx + cx(i)] - nxc;
      const double dy = s.b[1][by + cy(i)][bx + cx(i)] - nyc;
      dn += wtd(i) * ((double)cx(i) * dx + (double)cy(i) * dy);
    }
    dn *= 3.0;
    const double gx = s.gl[0][by][bx], gy = s.gl[1][by][bx];
    if constexpr (FORM == 6) {              // CSF-1: -kappa |G|^2 n div n
      const double k = -kappa * (gx * gx + gy * gy) * dn;
      fx = k * nxc;
      fy = k * nyc;
    } else {                                // CSF-2: -(sigma/2) G div n
      fx = -c.sigma_half_d * gx * dn;
      fy = -c.sigma_half_d * gy * dn;
    }
  }
  fxo = fx;
  fyo = fy;
}

// Everything the collision of an active node needs (FP64 arithmetic, FP32
// storage): the pulled flow populations and the node's moments.
struct NodeState {
  float f[9];
  float fx, fy, grx, gry, mu;
  double ux, uy, rho, P;
};

// Pull the stored flow populations for node (x, y) inside the domain
// (Eqs. 29 and 43, pull form).
template <bool WX, bool WY>
__device__ __forceinline__ void load_fp(const StepArgs& a, int x, int y, float* ft) {
  constexpr int wx = WX, wy = WY;
#define PULL_FP(I)                                               \
  {                                                              \
    int sl_;                                                     \
    const size_t b_ = src_base<I>(x, y, a.g, wx, wy, sl_);       \
    ft[I] = a.sin[b_ + (unsigned)((kPF + sl_) * 64)];            \
  }
  PULL_FP(0) PULL_FP(1) PULL_FP(2) PULL_FP(3) PULL_FP(4) PULL_FP(5) PULL_FP(6) PULL_FP(7) PULL_FP(8)
#undef PULL_FP
}

// Velocity (and, for active nodes, the rest of Eq. 37) at a node whose
// velocity-ring position is (uy_, ux_), from its pulled flow populations ft.
template <int FORM, bool FULL, class S>
__device__ __forceinline__ void velocity_from(const Lds<S>& s, const StepArgs& a, int uy_, int ux_, const float* ft,
                                              NodeState& ns) {
  double fx, fy;
  force_sf<FORM, S>(s, uy_, ux_, a.c, fx, fy);
  const double phid = s.phi[uy_ + 2][ux_ + 2];
  const double rho = rho_of(phid, a.c);
  fx += (rho - a.c.rho0_d) * a.c.gx_d;   // F_g = (rho - rho0) g   (Eq. 8)
  fy += (rho - a.c.rho0_d) * a.c.gy_d;
  double jx = 0.0, jy = 0.0;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const double fi = (double)ft[i];
    if (cx(i) != 0) jx += cx(i) * fi;
    if (cy(i) != 0) jy += cy(i) * fi;
  }
  const double inv_rho = rcp64(rho);
  const double ux = (3.0 * jx + 0.5 * fx) * inv_rho;   // Eq. (37)
  const double uy = (3.0 * jy + 0.5 * fy) * inv_rho;
  ns.ux = ux;
  ns.uy = uy;
  if constexpr (FULL) {
    const double gx = s.gl[0][uy_ + 1][ux_ + 1], gy = s.gl[1][uy_ + 1][ux_ + 1], lap = s.gl[2][uy_ + 1][ux_ + 1];
    const double grx = a.c.drho_half_d * gx, gry = a.c.drho_half_d * gy;   // grad rho = (rho1 - rho2)/2 grad phi
    ns.fx = (float)fx;
    ns.fy = (float)fy;
    ns.rho = rho;
    ns.grx = (float)grx;
    ns.gry = (float)gry;
    ns.mu = (float)chem_pot(phid, lap, a.c);
    double sumf = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) sumf += (double)ft[i];
    ns.P = sumf + (ux * grx + uy * gry) * (0.5 / 3.0);   // Eq. (37)
#pragma unroll
    for (int i = 0; i < 9; ++i) ns.f[i] = ft[i];
  }
}

// D_form = P_sf - p_h at velocity-ring position (uy_, ux_): the gradient
// terms each force form moves into its generalised pressure (Sec. II.B,
// Eq. 21 for CPF and PF; zero for STF-2 and CSF).  STF-1 takes
// -kappa |grad phi|^2, the value Eqs. (19) and (26) give (the sign printed
// with Eq. 17 contradicts them).  f0 = beta (1 - phi^2)^2.
template <int FORM, class S>
__device__ __forceinline__ double pressure_offset(const Lds<S>& s, int uy_, int ux_, const Phys& c) {
  const double phi = s.phi[uy_ + 2][ux_ + 2];
  const double gx = s.gl[0][uy_ + 1][ux_ + 1], gy = s.gl[1][uy_ + 1][ux_ + 1], lap = s.gl[2][uy_ + 1][ux_ + 1];
  const double kg2 = c.kappa_d * (gx * gx + gy * gy);
  const double om = (1.0 - phi) * (1.0 + phi);
  const double f0 = 0.25 * c.beta4_d * om * om;
  if constexpr (FORM == 0) return -kg2;
  else if constexpr (FORM == 2) return f0 - phi * chem_pot(phi, lap, c) - 0.5 * kg2;
  else if constexpr (FORM == 3) return f0 - 0.5 * kg2;
  else if constexpr (FORM == 4) return -0.5 * kg2;
  else if constexpr (FORM == 5) return c.kappa_d * phi * lap - 0.5 * kg2;
  else return 0.0;   // STF-2, CSF-1, CSF-2
}

__device__ __forceinline__ bool in_domain(int x, int y, const Grid& g) { return x >= 0 && x < g.nx && y >= 0 && y < g.ny; }

// Velocity-ring position k -> (uy_, ux_)
template <class S>
__device__ __forceinline__ void ring_pos(int k, int& uy_, int& ux_) {
  if (k < S::UW) { uy_ = 0; ux_ = k; }
  else if (k < 2 * S::UW) { uy_ = S::UH - 1; ux_ = k - S::UW; }
  else if (k < 2 * S::UW + S::TY) { uy_ = k - 2 * S::UW + 1; ux_ = 0; }
  else { uy_ = k - 2 * S::UW - S::TY + 1; ux_ = S::UW - 1; }
}

// Global position of ring position, wrapped on periodic axes; returns false
// when it lies beyond a wall (its velocity is then never read directly).
template <bool WX, bool WY>
__device__ __forceinline__ bool ring_global(int uy_, int ux_, int x0, int y0, const StepArgs& a, int& x, int& y) {
  x = x0 + ux_ - 1;
  y = y0 + uy_ - 1;
  if constexpr (WX) { if (x < 0 || x >= a.g.nx) return false; }
  else { x %= a.g.nx; if (x < 0) x += a.g.nx; }
  if constexpr (WY) { if (y < 0 || y >= a.g.ny) return false; }
  else { y %= a.g.ny; if (y < 0) y += a.g.ny; }
  return true;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Tile t is given to workgroup (t % per) * 8 + t / per, so every XCD
// sweeps one contiguous band of tiles (row-major) and the halos it shares
// with the previous tile and tile row are L2 hits.  Returns false for the
// padding workgroups past the last tile.
__device__ __forceinline__ bool xcd_tile(int ntx, int nty, int& tx, int& ty) {
  const int n = ntx * nty, per = (n + kXcds - 1) / kXcds;
  const int wg = blockIdx.x;
  const int t = (wg % kXcds) * per + wg / kXcds;
  if (t >= n) return false;
  ty = t / ntx;
  tx = t - ty * ntx;
  return true;
}

// c_i . v with the zero components of c_i dropped once the direction loop is
// unrolled (x + (-0.0) folds to x; 0 * x does not fold).
__device__ __forceinline__ double dotc(int i, double vx, double vy) {
  const double tx = cx(i) == 0 ? -0.0 : (cx(i) > 0 ? vx : -vx);
  const double ty = cy(i) == 0 ? -0.0 : (cy(i) > 0 ? vy : -vy);
  return tx + ty;
}
__device__ __forceinline__ float dotcf(int i, float vx, float vy) {
  const float tx = cx(i) == 0 ? -0.0f : (cx(i) > 0 ? vx : -vx);
  const float ty = cy(i) == 0 ? -0.0f : (cy(i) > 0 ? vy : -vy);
  return tx + ty;
}

// Pulled flow populations of a node of an interior tile (offsets v3, see
// node_offsets).
template <bool NT>
__device__ __forceinline__ void load_fp_tile(const float* tin, int rowe, const unsigned* v3, float* ft) {
#define PULL_FT(I) ft[I] = pull_tile<I, kPF + I, NT>(tin, rowe, v3);
  PULL_FT(0) PULL_FT(1) PULL_FT(2) PULL_FT(3) PULL_FT(4) PULL_FT(5) PULL_FT(6) PULL_FT(7) PULL_FT(8)
#undef PULL_FT
}

// Tiles of a periodic lattice that are not interior (the phi halo or a pull
// wraps): byte offsets, from the state array's base, of the columns x - 1,
// x, x + 1 (within a row) and of the rows y - 1, y, y + 1 around node (x, y)
// inside the domain, each wrapped once.  A pull of direction I reads column
// 1 - c_Ix of row 1 - c_Iy; the plane is a uniform constant, so a pull costs
// one vector add (the general path spends a wrap and a node index on each).
// Needs the whole array within 4 GiB (Grid::fast bit kFastWrap).
__device__ __forceinline__ void wrap_offsets(const Grid& g, int x, int y, unsigned* col, unsigned* row) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int X = x + k - 1, Y = y + k - 1;
    X = X < 0 ? X + g.nx : (X >= g.nx ? X - g.nx : X);
    Y = Y < 0 ? Y + g.ny : (Y >= g.ny ? Y - g.ny : Y);
    col[k] = 4u * (unsigned)((X >> 6) * kSegE + (X & 63));
    row[k] = 4u * (unsigned)Y * (unsigned)g.rowe;
  }
}

// Population plane P pulled in direction I by the node with wrapped offsets.
template <int I, int P, bool NT>
__device__ __forceinline__ float pull_wrap(const float* base, const unsigned* col, const unsigned* row) {
  const float* q = at(base + P * 64, row[1 - cy(I)] + col[1 - cx(I)]);
  if constexpr (NT) return ld_nt(q);
  else return *q;
}

template <bool NT>
__device__ __forceinline__ void load_fp_wrap(const float* base, const unsigned* col, const unsigned* row, float* ft) {
#define PULL_FW(I) ft[I] = pull_wrap<I, kPF + I, NT>(base, col, row);
  PULL_FW(0) PULL_FW(1) PULL_FW(2) PULL_FW(3) PULL_FW(4) PULL_FW(5) PULL_FW(6) PULL_FW(7) PULL_FW(8)
#undef PULL_FW
}

// A tile is interior when every position it reads (the phi halo reaches 3
// nodes past the tile) lies inside the domain: no wrap, mirror or bounce.
template <class S>
__device__ __forceinline__ bool interior_tile(int x0, int y0, const Grid& g) {
  return (g.fast & kFastInterior) && x0 >= 3 && y0 >= 3 && x0 + S::TX + 3 <= g.nx && y0 + S::TY + 3 <= g.ny;
}

// Wall term of Eq. (43) for a population leaving node (x, y) in direction
// I: true (and c_i . u_w) when x + c_i lies beyond a wall.
template <int I, bool WX, bool WY>
__device__ __forceinline__ bool wall_hit(int x, int y, const Grid& g, const Phys& c, double& cuw) {
  const int tx = x + cx(I), tyy = y + cy(I);
  bool hit = false;
  cuw = 0.0;
  if (WX && cx(I) != 0 && (tx < 0 || tx >= g.nx)) { hit = true; cuw = (double)cy(I) * (tx < 0 ? c.uw_lo_d : c.uw_hi_d); }
  if (WY && cy(I) != 0 && (tyy < 0 || tyy >= g.ny)) { hit = true; cuw = (double)cx(I) * (tyy < 0 ? c.uw_lo_d : c.uw_hi_d); }
  return hit;
}

// Collision results of one opposite pair (I, J = opp(I)) of both population
// sets, stored with the wall term applied (general tiles) or directly
// (interior and wrapped tiles: output origin tout, byte offset ob).
template <int I, bool DIRECT, bool WX, bool WY>
__device__ __forceinline__ void store_pair(const StepArgs& a, int x, int y, size_t on, float* tout, unsigned ob,
                                           double fpi, double fpj, double hpi, double hpj, double rho, double phid,
                                           double& d0sum) {
  constexpr int J = opp(I);
  if constexpr (!DIRECT) {
    double cuw;
    if (wall_hit<I, WX, WY>(x, y, a.g, a.c, cuw)) { fpi -= 2.0 * wtd(I) * rho * cuw; hpi -= 6.0 * wtd(I) * phid * cuw; }
    if (wall_hit<J, WX, WY>(x, y, a.g, a.c, cuw)) { fpj -= 2.0 * wtd(J) * rho * cuw; hpj -= 6.0 * wtd(J) * phid * cuw; }
  }
  const float hsi = (float)hpi, hsj = (float)hpj;
  d0sum += (double)hsi + (double)hsj;
  if constexpr (DIRECT) {
    st_nt(at(tout + (kPF + I) * 64, ob), (float)fpi);
    st_nt(at(tout + (kPF + J) * 64, ob), (float)fpj);
    st_nt(at(tout + (kPH + I) * 64, ob), hsi);
    st_nt(at(tout + (kPH + J) * 64, ob), hsj);
  } else {
    a.sout[on + (unsigned)((kPF + I) * 64)] = (float)fpi;
    a.sout[on + (unsigned)((kPF + J) * 64)] = (float)fpj;
    a.sout[on + (unsigned)((kPH + I) * 64)] = hsi;
    a.sout[on + (unsigned)((kPH + J) * 64)] = hsj;
  }
}


// The thread index of a tile body.  A persistent kernel runs the body in a
// loop (LOOPED); there the compiler would hoist every value derived from the
// index out of the loop and hold it across the whole body (spills at the
// 128 VGPRs of four waves per SIMD).  An index it cannot see through is
// recomputed per tile instead.
template <bool LOOPED>
__device__ __forceinline__ int tile_tid() {
  int t = threadIdx.x;
  if constexpr (LOOPED) asm volatile("" : "+v"(t));
  return t;
}

// Addressing paths of a tile: general (wraps, mirrors and bounce-back per
// pull), interior (see interior_tile) and wrapped (periodic lattices, see
// wrap_offsets).  All three store the same values.
constexpr int kPathGeneral = 0, kPathInterior = 1, kPathWrapped = 2;

// One tile of the step (or of the moments): the whole per-node update of
// a1-a12.  PATH: one of the addressing paths above; the moments take the
// general one.
template <class S, int FORM, bool MOMENTS, int BC, int PATH, bool LOOPED>
__device__ __forceinline__ void tile_impl(Lds<S>& s, const StepArgs& a, const MomentArgs& m, int tile_x, int tile_y) {
  constexpr bool FAST = PATH == kPathInterior, WRAP = PATH == kPathWrapped, DIRECT = FAST || WRAP;
  static_assert(!(DIRECT && MOMENTS), "the moments use the general path");
  static_assert(!WRAP || BC == 0, "the wrapped path is for periodic lattices");
  constexpr bool WX = (BC & 1) != 0, WY = (BC & 2) != 0;   // walled axes (compile time)
  const int tid = tile_tid<LOOPED>();
  constexpr int PW = S::PW, PH = S::PH, NT = S::NT;
  const int x0 = tile_x * S::TX, y0 = tile_y * S::TY;
  const int lx = tid & (S::TX - 1), ty = tid / S::TX;   // one node per thread
  const Grid& g = a.g;
  const Phys& c = a.c;
  const int uy_ = ty + 1, ux_ = lx + 1;             // velocity-ring coordinates of this node
  int x, y;
  bool valid, act;
  const float* tin = nullptr;   // interior tiles: input origin (node (tile_xo(x0), y0 - 2))
  float* tout = nullptr;        // interior tiles: output origin (node (x0, y0))
  if constexpr (FAST) {
    x = x0 + lx;
    y = y0 + ty;
    valid = act = true;
    tin = a.sin + nbase(g, tile_xo(x0), y0 - 2);
    tout = a.sout + nbase(g, x0, y0);
  } else {
    valid = ring_global<WX, WY>(uy_, ux_, x0, y0, a, x, y);
    act = (x0 + lx < g.nx) && (y0 + ty < g.ny);
    if constexpr (WRAP) tout = a.sout;   // wrapped offsets are from the array base
  }
  const size_t on = nbase(g, x, y);   // general path: plane 0 of this node (valid nodes)

  // This node's flow populations are pulled after the ring velocities (the
  // ring threads would otherwise hold both sets of registers at once).  The
  // ring threads request their ring node's populations right after staging
  // the order parameter, so those loads are in flight through the first
  // barrier and the stencil stage: nothing waits for them before the ring's
  // velocities.
  float ft[9], h[9];
  float j0 = 0.f, j1 = 0.f;
  // Only ring threads define these.  The others start from a kernel
  // argument, not a constant: with a constant there the compiler moves the
  // FP64 conversions of the ring values up to their loads, and the ring
  // threads then wait for those loads as soon as they are issued.
  float rft[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) rft[i] = c.gx;
  int ruy = 0, rux = 0;
  bool ring_ok = true;   // general path: the ring position is not beyond a wall
  // Stage A: phi tile with a 3-node halo (periodic wrap / even reflection at walls, Sec. IV)
  if constexpr (FAST) {
    // every load of a thread in flight before any is stored
    const double* tphi = a.phi + ((long long)(y0 - 3) * g.pitch + (x0 - 3));
    double pv[S::NPHI];
#pragma unroll
    for (int j = 0; j < S::NPHI; ++j) {
      const int k = tid + j * NT, py = k / PW, px = k - py * PW;
      pv[j] = (j == 0 || k < PH * PW) ? *at(tphi, (unsigned)(py * g.pitch + px) * 8u) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < S::NPHI; ++j) {
      const int k = tid + j * NT, py = k / PW, px = k - py * PW;
      if (j == 0 || k < PH * PW) s.phi[py][px] = pv[j];
    }
    if constexpr (!MOMENTS) {
      if (tid < S::NRING) {
        ring_pos<S>(tid, ruy, rux);
        unsigned rv[3];
        node_offsets(g, x0, rux - 1, ruy - 1, rv);
        load_fp_tile<false>(tin, g.rowe, rv, rft);
      }
    }
  } else {
    // the same order as on interior tiles: the phi loads, the stores, then
    // the ring's pulls, which stay in flight through the stencil stage
    double pv[S::NPHI];
#pragma unroll
    for (int j = 0; j < S::NPHI; ++j) {
      const int k = tid + j * NT, py = k / PW, px = k - py * PW;
      pv[j] = (j == 0 || k < PH * PW)
                  ? a.phi[(unsigned)(halo_coord<WY>(y0 + py - 3, g.ny) * g.pitch + halo_coord<WX>(x0 + px - 3, g.nx))]
                  : 0.0;
    }
#pragma unroll
    for (int j = 0; j < S::NPHI; ++j) {
      const int k = tid + j * NT, py = k / PW, px = k - py * PW;
      if (j == 0 || k < PH * PW) s.phi[py][px] = pv[j];
    }
    if constexpr (!MOMENTS) {
      if (tid < S::NRING) {
        ring_pos<S>(tid, ruy, rux);
        int rx, ry;
        ring_ok = ring_global<WX, WY>(ruy, rux, x0, y0, a, rx, ry);
        if constexpr (WRAP) {
          unsigned rc[3], rr[3];
          wrap_offsets(g, rx, ry, rc, rr);
          load_fp_wrap<false>(a.sin, rc, rr, rft);
        } else if (ring_ok) {
          load_fp<WX, WY>(a, rx, ry, rft);
        }
      }
    }
  }
  __syncthreads();

  stage_b<FORM, S>(s, tid, c);
  __syncthreads();

  // Stage C: velocities of the ring (step only), then of this node.  On
  // interior tiles this node's pulls are issued first for the CPF and PF
  // forms, so their latency overlaps the ring's work (measured: no gain for
  // the CSF forms, and the stress forms need those registers for the ring).
  constexpr bool kEarlyOwn = FAST && FORM >= 2 && FORM <= 5;
  // The CPF, PF and stress forms also request their h and (phi u) pulls
  // before the last barrier (measured: -1 to -6 us; the CSF forms gain
  // nothing).
  constexpr bool kEarlyH = FAST && FORM <= 5;
  unsigned v3[3] = {0u, 0u, 0u};
  if constexpr (FAST) node_offsets(g, x0, lx, ty, v3);
  // The last wave's own pulls (the tile's bottom rows) are cached loads: the
  // velocity ring of the next tile row reads those lines again (measured:
  // 0.8 B/node less HBM reading).  The branch is uniform per wave.
  const bool own_cached = (tid >> 6) == (NT >> 6) - 1;
  if constexpr (kEarlyOwn) {
    if (own_cached) load_fp_tile<false>(tin, g.rowe, v3, ft);
    else load_fp_tile<true>(tin, g.rowe, v3, ft);
  }
  if constexpr (!MOMENTS) {
    if (tid < S::NRING) {
      if (FAST || ring_ok) {
        NodeState rs;
        velocity_from<FORM, false, S>(s, a, ruy, rux, rft, rs);
        const double ph = s.phi[ruy + 2][rux + 2];
        s.q[0][ruy][rux] = (float)(ph * rs.ux);
        s.q[1][ruy][rux] = (float)(ph * rs.uy);
      }
    }
  }
  // wrapped path: this node's offsets (formed after the ring's work, which
  // would otherwise hold them as well)
  unsigned wc[3] = {0u, 0u, 0u}, wr[3] = {0u, 0u, 0u};
  if constexpr (WRAP) wrap_offsets(g, x, y, wc, wr);
  NodeState n;
  if (valid) {
    if constexpr (WRAP) load_fp_wrap<true>(a.sin, wc, wr, ft);
    else if constexpr (!FAST) load_fp<WX, WY>(a, x, y, ft);
    else if constexpr (!kEarlyOwn) {
      if (own_cached) load_fp_tile<false>(tin, g.rowe, v3, ft);
      else load_fp_tile<true>(tin, g.rowe, v3, ft);
    }
    velocity_from<FORM, true, S>(s, a, uy_, ux_, ft, n);
    if constexpr (!MOMENTS) {
      const double ph = s.phi[uy_ + 2][ux_ + 2];
      s.q[0][uy_][ux_] = (float)(ph * n.ux);
      s.q[1][uy_][ux_] = (float)(ph * n.uy);
    }
  }
  if constexpr (MOMENTS) {
    if (act) {
      const long long om = (long long)y * g.nx + x;
      if (m.phi) m.phi[om] = (float)s.phi[ty + 3][lx + 3];
      if (m.rho) m.rho[om] = (float)n.rho;
      if (m.ux) m.ux[om] = (float)n.ux;
      if (m.uy) m.uy[om] = (float)n.uy;
      if (m.p) m.p[om] = (float)n.P;
      if (m.ph) m.ph[om] = (float)(n.P - pressure_offset<FORM, S>(s, uy_, ux_, c));
    }
    return;
  } else {
    if constexpr (kEarlyH) {
      h[1] = pull_tile<1, kPH + 1, true>(tin, g.rowe, v3);
      h[2] = pull_tile<2, kPH + 2, true>(tin, g.rowe, v3);
      h[3] = pull_tile<3, kPH + 3, true>(tin, g.rowe, v3);
      h[4] = pull_tile<4, kPH + 4, true>(tin, g.rowe, v3);
      h[5] = pull_tile<5, kPH + 5, true>(tin, g.rowe, v3);
      h[6] = pull_tile<6, kPH + 6, true>(tin, g.rowe, v3);
      h[7] = pull_tile<7, kPH + 7, true>(tin, g.rowe, v3);
      h[8] = pull_tile<8, kPH + 8, true>(tin, g.rowe, v3);
      j0 = pull_tile<0, kPJ, true>(tin, g.rowe, v3);
      j1 = pull_tile<0, kPJ + 1, true>(tin, g.rowe, v3);
    }
    __syncthreads();
    if (!act) return;
    if constexpr (FAST && !kEarlyH) {
      h[1] = pull_tile<1, kPH + 1, true>(tin, g.rowe, v3);
      h[2] = pull_tile<2, kPH + 2, true>(tin, g.rowe, v3);
      h[3] = pull_tile<3, kPH + 3, true>(tin, g.rowe, v3);
      h[4] = pull_tile<4, kPH + 4, true>(tin, g.rowe, v3);
      h[5] = pull_tile<5, kPH + 5, true>(tin, g.rowe, v3);
      h[6] = pull_tile<6, kPH + 6, true>(tin, g.rowe, v3);
      h[7] = pull_tile<7, kPH + 7, true>(tin, g.rowe, v3);
      h[8] = pull_tile<8, kPH + 8, true>(tin, g.rowe, v3);
      j0 = pull_tile<0, kPJ, true>(tin, g.rowe, v3);
      j1 = pull_tile<0, kPJ + 1, true>(tin, g.rowe, v3);
    } else if constexpr (WRAP) {
      h[1] = pull_wrap<1, kPH + 1, true>(a.sin, wc, wr);
      h[2] = pull_wrap<2, kPH + 2, true>(a.sin, wc, wr);
      h[3] = pull_wrap<3, kPH + 3, true>(a.sin, wc, wr);
      h[4] = pull_wrap<4, kPH + 4, true>(a.sin, wc, wr);
      h[5] = pull_wrap<5, kPH + 5, true>(a.sin, wc, wr);
      h[6] = pull_wrap<6, kPH + 6, true>(a.sin, wc, wr);
      h[7] = pull_wrap<7, kPH + 7, true>(a.sin, wc, wr);
      h[8] = pull_wrap<8, kPH + 8, true>(a.sin, wc, wr);
      j0 = pull_wrap<0, kPJ, true>(a.sin, wc, wr);
      j1 = pull_wrap<0, kPJ + 1, true>(a.sin, wc, wr);
    } else if constexpr (!FAST) {
      constexpr int wx = WX, wy = WY;
#define PULL_HG(I)                                                 \
  {                                                                \
    int sl_;                                                       \
    const size_t b_ = src_base<I>(x, y, g, wx, wy, sl_);           \
    h[I] = a.sin[b_ + (unsigned)((kPH + sl_) * 64)];               \
  }
      PULL_HG(1) PULL_HG(2) PULL_HG(3) PULL_HG(4) PULL_HG(5) PULL_HG(6) PULL_HG(7) PULL_HG(8)
#undef PULL_HG
      j0 = a.sin[on + (unsigned)(kPJ * 64)];
      j1 = a.sin[on + (unsigned)((kPJ + 1) * 64)];
    }

    const int py = uy_ + 2, px = ux_ + 2;
    const double phid = s.phi[py][px];
    // div(phi u) (Eq. 41) from the node field q = phi u; beyond a wall the
    // ghost velocity is 2 u_w - u(mirror) with phi mirrored (A9), i.e.
    // q_ghost = 2 u_w phi(mirror) - q(mirror) along the wall, -q(mirror) across.
    float dqf = 0.f;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      int qy = uy_ + cy(i), qx = ux_ + cx(i);
      float vx, vy;
      if constexpr (FAST) {
        vx = s.q[0][qy][qx];
        vy = s.q[1][qy][qx];
      } else {
        const int nxg = x + cx(i), nyg = y + cy(i);
        const bool gx_ = WX && (nxg < 0 || nxg >= g.nx);
        const bool gy_ = WY && (nyg < 0 || nyg >= g.ny);
        if (gx_) qx = ux_;
        if (gy_) qy = uy_;
        vx = s.q[0][qy][qx];
        vy = s.q[1][qy][qx];
        if (gx_ || gy_) {   // a free-slip wall mirrors: only the normal component flips
          const float phm = (float)s.phi[qy + 2][qx + 2];
          if (gx_) { vx = -vx; if (!g.slip_x) vy = 2.f * (nxg < 0 ? c.uw_lo : c.uw_hi) * phm - vy; }
          if (gy_) { if (!g.slip_y) vx = 2.f * (nyg < 0 ? c.uw_lo : c.uw_hi) * phm - vx; vy = -vy; }
        }
      }
      dqf += wt(i) * dotcf(i, vx, vy);
    }
    const double dq = 3.0 * (double)dqf;
    const double qx = phid * n.ux, qy = phid * n.uy;
    const double dtx = qx - (double)j0, dty = qy - (double)j1;   // explicit-Euler d_t(phi u) (A4)
    // this node from tout: interior tiles from the tile origin, wrapped ones from the array base
    const unsigned ob = WRAP ? wr[1] + wc[1] : 4u * (unsigned)(ty * g.rowe + lx);
    if constexpr (DIRECT) {
      st_nt(at(tout + kPJ * 64, ob), (float)qx);
      st_nt(at(tout + (kPJ + 1) * 64, ob), (float)qy);
    } else {
      a.sout[on + (unsigned)(kPJ * 64)] = (float)qx;
      a.sout[on + (unsigned)((kPJ + 1) * 64)] = (float)qy;
    }

    if (!(isfinite(n.ux) && isfinite(n.uy) && isfinite(phid))) atomicOr(a.status, 1);

    const double tau_f = 0.5 + 3.0 * mu_of(phid, c) * rcp64(n.rho);   // A6
    const double omf = rcp64(tau_f), cff = 1.0 - 0.5 * omf;
    const double omh = c.inv_tau_h_d, cfh = 1.0 - 0.5 * omh;
    const double usq = n.ux * n.ux + n.uy * n.uy;

    // Order-parameter collision, Eq. (30) with h^eq of Eq. (32) and H_i of
    // Eq. (36), factored per node:  h_i^+ = (1 - 1/tau_h) h_i + w_i [G0 + 3 c_i.V]
    // with G0 = eta mu / tau_h + (1 - 1/(2 tau_h)) A_H div(phi u) and
    // V = phi u / tau_h + (1 - 1/(2 tau_h)) d_t(phi u).
    const double G0 = omh * c.eta_d * (double)n.mu + cfh * (c.a_h_d * dq);
    const double Vx = omh * qx + cfh * dtx, Vy = omh * qy + cfh * dty;
    const double keep_h = 1.0 - omh;

    // Flow collision, Eq. (29) with f^eq of Eq. (31) and F_i of Eq. (35)
    // (reading A1), factored per node.  With s_i = 3 c.u + 4.5 (c.u)^2 - 1.5 u^2,
    // F = F_sf + F_g and grad rho:
    //   f_i^+ = (1 - 1/tau_f) f_i + w_i [K0 + k c.F + s_i (K1 + k c.F + k c.grad(rho)/3)],
    //   k = 1 - 1/(2 tau_f), K0 = P/tau_f - k u.F,
    //   K1 = rho/(3 tau_f) - k u.F - k u.grad(rho)/3.
    // Directions come in opposite pairs (c_J = -c_I): s = e +- o with the
    // even part e = 4.5 (c.u)^2 - 1.5 u^2 and the odd part o = 3 c.u, so
    // f_I^+, f_J^+ = keep f + w (Se +- Qo) with Se = K0 + e K1 + o d,
    // Qo = c.kF + e d + o K1, d = c.kF + c.kG.  Likewise h_I^+, h_J^+ =
    // keep h + w (G0 +- 3 c.V).
    const double fx = (double)n.fx, fy = (double)n.fy, grx = (double)n.grx, gry = (double)n.gry;
    const double uF = n.ux * fx + n.uy * fy, uG = n.ux * grx + n.uy * gry;
    const double K0 = omf * n.P - cff * uF;
    const double K1 = omf * n.rho * (1.0 / 3.0) - cff * uF - cff * uG * (1.0 / 3.0);
    const double kFx = cff * fx, kFy = cff * fy;
    const double kFGx = kFx + cff * grx * (1.0 / 3.0), kFGy = kFy + cff * gry * (1.0 / 3.0);
    const double keep_f = 1.0 - omf, m15usq = -1.5 * usq;
    double d0sum = 0.0;   // sum of the stored h_i^+ (i >= 1)
    {
      const double fp0 = keep_f * (double)n.f[0] + wtd(0) * fma(m15usq, K1, K0);
      if constexpr (DIRECT) st_nt(at(tout + kPF * 64, ob), (float)fp0);
      else a.sout[on + (unsigned)(kPF * 64)] = (float)fp0;
    }
#define COLLIDE_PAIR(I)                                                                        \
  {                                                                                            \
    constexpr int J_ = opp(I);                                                                 \
    const double cu = dotc(I, n.ux, n.uy);                                                     \
    const double e = fma(4.5 * cu, cu, m15usq), od = 3.0 * cu;                                 \
    const double cF = dotc(I, kFx, kFy), d = dotc(I, kFGx, kFGy);                              \
    const double Se = fma(od, d, fma(e, K1, K0)), Qo = fma(od, K1, fma(e, d, cF));             \
    const double wS = wtd(I) * Se, wQ = wtd(I) * Qo;                                           \
    const double fpi = fma(keep_f, (double)n.f[I], wS + wQ);                                   \
    const double fpj = fma(keep_f, (double)n.f[J_], wS - wQ);                                  \
    const double wG = wtd(I) * G0, t = (3.0 * wtd(I)) * dotc(I, Vx, Vy);                      \
    const double hpi = fma(keep_h, (double)h[I], wG + t);                                      \
    const double hpj = fma(keep_h, (double)h[J_], wG - t);                                     \
    store_pair<I, DIRECT, WX, WY>(a, x, y, on, tout, ob, fpi, fpj, hpi, hpj, n.rho, phid, d0sum); \
  }
    COLLIDE_PAIR(1) COLLIDE_PAIR(2) COLLIDE_PAIR(5) COLLIDE_PAIR(6)
#undef COLLIDE_PAIR
    // slot 0 holds d0 = h_0^+ - phi.  The collision conserves sum_i h_i = phi
    // (Eqs. 32 and 36), so d0 = -sum_{i>=1} h_i^+ exactly; forming it from
    // the stored values makes the update of phi conservative.
    if constexpr (DIRECT) st_nt(at(tout + kPH * 64, ob), (float)(-d0sum));
    else a.sout[on + (unsigned)(kPH * 64)] = (float)(-d0sum);
  }
}

// One tile on the best path its position allows.  WRAP_EDGES: the edge
// tiles of a periodic lattice take the wrapped path (when the array allows
// it) instead of the general one.  Measured on a 2048^2 lattice, where 7 %
// of the tiles are edge tiles, the wrapped path makes the step 1.5 % slower
// (its non-temporal stores; with plain stores it is even, and the batched
// step, where it pays, loses 3-7 % with them), so a single lattice keeps
// the general path on its edge.
template <class S, int FORM, bool MOMENTS, int BC, bool LOOPED, bool WRAP_EDGES = false>
__device__ __forceinline__ void fused_tile(Lds<S>& s, const StepArgs& a, const MomentArgs& m, int tile_x, int tile_y) {
  if constexpr (!MOMENTS) {
    if (interior_tile<S>(tile_x * S::TX, tile_y * S::TY, a.g)) {
      tile_impl<S, FORM, false, BC, kPathInterior, LOOPED>(s, a, m, tile_x, tile_y);
      return;
    }
    if constexpr (BC == 0 && WRAP_EDGES) {
      if (a.g.fast & kFastWrap) {
        tile_impl<S, FORM, false, BC, kPathWrapped, LOOPED>(s, a, m, tile_x, tile_y);
        return;
      }
    }
  }
  tile_impl<S, FORM, MOMENTS, BC, kPathGeneral, LOOPED>(s, a, m, tile_x, tile_y);
}

// phi^{n+1}(x) = phi^n(x) + d0(x) + sum_{i>=1} h_i^+(x - c_i)   (Eq. 37,
// phi = sum h_i), from the state array just written (snew).  Both paths sum
// in the same order.
template <class S, int BC, int PATH>
__device__ __forceinline__ void phi_tile_impl(const float* __restrict__ snew, const double* phi_in, double* phi_out,
                                              const Grid& g,
                                              int tile_x, int tile_y) {
  constexpr int wx = (BC & 1) != 0, wy = (BC & 2) != 0;
  const int lx = threadIdx.x & (S::TX - 1), ty = threadIdx.x / S::TX;
  const int x = tile_x * S::TX + lx, y = tile_y * S::TY + ty;
  if (x >= g.nx || y >= g.ny) return;
  double sum;
  if constexpr (PATH == kPathWrapped) {
    unsigned col[3], row[3];
    wrap_offsets(g, x, y, col, row);
    sum = (double)pull_wrap<0, kPH, true>(snew, col, row);
    sum += (double)pull_wrap<1, kPH + 1, true>(snew, col, row);
    sum += (double)pull_wrap<2, kPH + 2, true>(snew, col, row);
    sum += (double)pull_wrap<3, kPH + 3, true>(snew, col, row);
    sum += (double)pull_wrap<4, kPH + 4, true>(snew, col, row);
    sum += (double)pull_wrap<5, kPH + 5, true>(snew, col, row);
    sum += (double)pull_wrap<6, kPH + 6, true>(snew, col, row);
    sum += (double)pull_wrap<7, kPH + 7, true>(snew, col, row);
    sum += (double)pull_wrap<8, kPH + 8, true>(snew, col, row);
  } else if constexpr (PATH == kPathInterior) {
    const float* tin = snew + nbase(g, tile_xo(tile_x * S::TX), tile_y * S::TY - 2);
    unsigned v3[3];
    node_offsets(g, tile_x * S::TX, lx, ty, v3);
    sum = (double)pull_tile<0, kPH, true>(tin, g.rowe, v3);
    sum += (double)pull_tile<1, kPH + 1, true>(tin, g.rowe, v3);
    sum += (double)pull_tile<2, kPH + 2, true>(tin, g.rowe, v3);
    sum += (double)pull_tile<3, kPH + 3, true>(tin, g.rowe, v3);
    sum += (double)pull_tile<4, kPH + 4, true>(tin, g.rowe, v3);
    sum += (double)pull_tile<5, kPH + 5, true>(tin, g.rowe, v3);
    sum += (double)pull_tile<6, kPH + 6, true>(tin, g.rowe, v3);
    sum += (double)pull_tile<7, kPH + 7, true>(tin, g.rowe, v3);
    sum += (double)pull_tile<8, kPH + 8, true>(tin, g.rowe, v3);
  } else {
    sum = (double)snew[nbase(g, x, y) + (unsigned)(kPH * 64)];
#define PULL_PH(I)                                               \
  {                                                              \
    int sl_;                                                     \
    const size_t b_ = src_base<I>(x, y, g, wx, wy, sl_);         \
    sum += (double)snew[b_ + (unsigned)((kPH + sl_) * 64)];      \
  }
    PULL_PH(1) PULL_PH(2) PULL_PH(3) PULL_PH(4) PULL_PH(5) PULL_PH(6) PULL_PH(7) PULL_PH(8)
#undef PULL_PH
  }
  // phi_in may be phi_out (in place): a thread reads and writes only its node
  phi_out[(long long)y * g.pitch + x] = phi_in[(long long)y * g.pitch + x] + sum;
}

// WRAP_EDGES as for fused_tile (the single-lattice pass is 3 % slower with it).
template <class S, int BC, bool WRAP_EDGES = false>
__device__ __forceinline__ void phi_tile(const float* snew, const double* phi_in, double* phi_out, const Grid& g,
                                         int tile_x, int tile_y) {
  if (interior_tile<S>(tile_x * S::TX, tile_y * S::TY, g))
    phi_tile_impl<S, BC, kPathInterior>(snew, phi_in, phi_out, g, tile_x, tile_y);
  else if (WRAP_EDGES && BC == 0 && (g.fast & kFastWrap))
    phi_tile_impl<S, BC, kPathWrapped>(snew, phi_in, phi_out, g, tile_x, tile_y);
  else
    phi_tile_impl<S, BC, kPathGeneral>(snew, phi_in, phi_out, g, tile_x, tile_y);
}

// Tile shapes by index (kShapeTX/kShapeTY in lbm_internal.hpp).
using S0 = Shape<kShapeTX[0], kShapeTY[0]>;
using S1 = Shape<kShapeTX[1], kShapeTY[1]>;
using S2 = Shape<kShapeTX[2], kShapeTY[2]>;
using S3 = Shape<kShapeTX[3], kShapeTY[3]>;

}  // namespace

}  // namespace pflbm
