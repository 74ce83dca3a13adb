// Internal declarations shared by the HIP kernels and the C-ABI host code.
//
// D2Q9 lattice of arXiv:2012.14729, Sec. III (Eq. 34 and the weights below
// it), stored as constexpr functions so fully unrolled loops fold them into
// immediates.  Device state of one lattice (x fastest, pitch = nx rounded up
// to 64):
//   S[2]  FP32 ping-pong state arrays of 20 planes, interleaved in row
//         segments of 64 nodes: element (plane p, x, y) lies at
//         ((y * ncx + x / 64) * 20 + p) * 64 + x % 64  (ncx = pitch / 64), so
//         the 20 values of a 64-node row segment are one 5120-byte run.
//         planes 0-8   f_i (post-collision)
//         planes 9-17  h_i (post-collision); plane 9 holds d0 = h_0^+ - phi
//         planes 18-19 (phi u) of the step that stored them
//   phi   FP64 plane (pitch * ny), updated in place
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pflbm {

__host__ __device__ constexpr int cx(int i) { return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0); }
__host__ __device__ constexpr int cy(int i) { return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0); }
__host__ __device__ constexpr float wt(int i) { return i == 0 ? 4.0f / 9.0f : (i < 5 ? 1.0f / 9.0f : 1.0f / 36.0f); }
__host__ __device__ constexpr double wtd(int i) { return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : (i < 5 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5); }
// direction with the x (mirror_x) or y (mirror_y) component of c_i reversed
__host__ __device__ constexpr int dir_of(int x, int y) {
  return x == 0 ? (y == 0 ? 0 : (y > 0 ? 2 : 4)) : (x > 0 ? (y == 0 ? 1 : (y > 0 ? 5 : 8)) : (y == 0 ? 3 : (y > 0 ? 6 : 7)));
}
__host__ __device__ constexpr int mirror_x(int i) { return dir_of(-cx(i), cy(i)); }
__host__ __device__ constexpr int mirror_y(int i) { return dir_of(cx(i), -cy(i)); }

constexpr int kNPL = 20;  // planes of a state array
constexpr int kPF = 0, kPH = 9, kPJ = 18;   // first plane of f, h, J
constexpr int kSegE = kNPL * 64;   // elements of one interleaved row segment

// Tile shapes of the fused and order-parameter kernels (TX x TY nodes, one
// node per thread), by index: 0 is the single-lattice shape, all four are
// candidates of the batched step's tuner.
constexpr int kNumShapes = 4;
constexpr int kShapeTX[kNumShapes] = {64, 32, 32, 64};
constexpr int kShapeTY[kNumShapes] = {8, 16, 8, 4};

// Per-simulation physical constants in the form the kernels use.
struct Phys {
  float rho_a, rho_b;     // rho(phi) = rho_a + rho_b phi      (Eq. 9)
  float mu_a, mu_b;       // mu(phi)  = mu_a + mu_b phi        (Eq. 10)
  float beta4, kappa;     // 4 beta, kappa                      (Eq. 6)
  float sigma_half;       // sigma / 2 (CSF-2)
  float eps2;             // eps_n^2 (CSF normal regulariser)
  float eta;              // M / (cs^2 (tau_h - 1/2))
  float a_h;              // 3 tau_2 / (tau_h tau_1)            (Eq. 36)
  float inv_tau_h;        // 1 / tau_h
  float gx, gy, rho0;     // F_g = (rho - rho0) g
  float uw_lo, uw_hi;     // wall speeds
  int wall_x, wall_y;
  double beta4_d, kappa_d, sigma_half_d, eps2_d;   // FP64 copies for the stencil stages
  double rho2_d, drho_half_d, mu2_d, dmu_half_d;   // rho = rho2 + (rho1-rho2)(1+phi)/2, same for mu
  double eta_d, a_h_d, inv_tau_h_d, gx_d, gy_d, rho0_d, uw_lo_d, uw_hi_d;
};

struct Grid {
  int nx, ny, pitch;
  int ncx;                // 64-node row segments per row (pitch / 64)
  long long ps;           // nodes of a padded plane (pitch * ny)
  int rowe;               // elements of one row of a state array (ncx * 20 * 64)
  int fast;               // addressing paths allowed (kFastInterior | kFastWrap)
  int slip_x, slip_y;     // the walls of that axis are free-slip (specular), not no-slip
};

// Grid::fast bits.  kFastInterior: interior tiles address from a tile
// origin.  kFastWrap: the other tiles of a periodic lattice address with
// 32-bit byte offsets from the state array's base, which needs the array
// within 4 GiB (fast_bits below).
constexpr int kFastInterior = 1, kFastWrap = 2;
__host__ __device__ constexpr int fast_bits(long long plane_nodes) {
  return kFastInterior | ((long long)kNPL * plane_nodes * 4 <= 0xffffffffLL ? kFastWrap : 0);
}

// Element index of plane 0 of node (x, y) in a state array, 64-bit (a state
// array may hold more than 2^32 elements; the segment index y ncx + x / 64
// stays below 2^31 because ps < 2^31 is validated); plane p of the node is
// 64 p elements further.
__host__ __device__ __forceinline__ size_t nbase(const Grid& g, int x, int y) {
  return (size_t)(unsigned)(y * g.ncx + (x >> 6)) * (size_t)kSegE + (size_t)(x & 63);
}

struct StepArgs {
  const float* sin;       // state array holding the current step
  float* sout;            // state array receiving the next step
  const double* phi;      // order parameter (read by the fused kernel, updated by k_phi)
  int* status;            // divergence flag
  Grid g;
  Phys c;
};

struct MomentArgs {
  float* phi;
  float* rho;
  float* ux;
  float* uy;
  float* p;
  float* ph;   // hydrodynamic pressure p_h = P_sf - D_form (Sec. II.B)
};

// Records the thread-local message returned by lbm_last_error(); returns code.
int set_error(int code, const char* fmt, ...);

}  // namespace pflbm
struct lbm_params;
namespace pflbm {
// Kernel constants of a problem statement (lbm_api.hip).
Phys derive_phys(const lbm_params* p, double rho0);

}  // namespace pflbm
struct lbm_sim;
namespace pflbm {
// Read access to a single lattice's current state (lbm_api.hip).
struct SimView {
  const float* s;     // state array of the current step (layout above)
  const double* phi;  // order parameter (current)
  Grid g;
};
int sim_params(const lbm_sim* s, lbm_params* out);
Phys sim_phys(const lbm_sim* s);
int sim_view(const lbm_sim* s, SimView* v);

// kernel launchers (lbm_kernels.hip); each returns the launch error code.
// t0, t1 (both or neither): events that take the kernel's own start and stop
// times from its dispatch.
hipError_t launch_fused(int form, int shape, const StepArgs& a, hipStream_t s, hipEvent_t t0 = nullptr,
                        hipEvent_t t1 = nullptr);
hipError_t launch_moments(int form, const StepArgs& a, const MomentArgs& m, hipStream_t s);
// phi_out = phi_in + d0 + sum of the pulled h (phi_out may be phi_in: in place)
hipError_t launch_phi(const float* snew, const double* phi_in, double* phi_out, const Grid& g, int wall_x, int wall_y,
                      int shape, hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t launch_init(const float* phi0, const float* ux0, const float* uy0, float* s_tmp, float* s0, double* phi,
                       const Grid& g, const Phys& c, hipStream_t s);
// sum of the phi plane: at most npartial (and one per 256 nodes) partial sums, then one
hipError_t launch_phi_sum(const double* phi, const Grid& g, double* partial, int npartial, double* out,
                          hipStream_t s);
hipError_t launch_fill_int(int* p, int value, int n, hipStream_t s);
// njobs (<= 3) copies of bytes[k] from src[k] to dst[k], then zero_bytes of
// zeros at `zero` (nullable), as one launch; sizes multiples of 4 bytes.
hipError_t launch_copies(const void* const* src, void* const* dst, const size_t* bytes, int njobs, void* zero,
                         size_t zero_bytes, hipStream_t s);

}  // namespace pflbm
