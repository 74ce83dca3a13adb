// HIP kernels (gfx950, wave64) of the phase-field lattice Boltzmann step of
// arXiv:2012.14729.
//
// One time step is two launches:
//   k_fused<FORM>  pull-stream f and h (with bounce-back), compute phi
//                  stencils, mu_phi, the interfacial force, u, P, div(phi u),
//                  d_t(phi u), collide both populations and store them.
//   k_phi          phi^{n+1} = phi^n + d0 + sum_{i>=1} h_i pulled, in FP64.
//
// The fused kernel works on TX x TY tiles, one node per thread (the tile
// shape is a template parameter: 64x8 for single lattices, a choice of shapes
// for the batched step).  The order parameter is staged in LDS with a 3-node
// halo (FP64); second-level stencil fields live on the 2-node ring, the
// velocity on the 1-node ring.  Only nearest-neighbour pulls touch
// HBM; everything with a wider footprint comes from LDS.  The state arrays
// interleave their 20 planes in 64-node row segments (lbm_internal.hpp), so a
// wavefront's loads and stores of one row segment form one contiguous run.
#include <hip/hip_ext.h>

#include "lbm_tile.hpp"

namespace pflbm {

namespace {
template <class S, int FORM, bool MOMENTS, int BC>
__global__ __launch_bounds__(S::NT) __attribute__((amdgpu_waves_per_eu(4))) void k_fused(StepArgs a, MomentArgs m) {
  __shared__ Lds<S> s;
  int tile_x, tile_y;
  if (!xcd_tile((a.g.nx + S::TX - 1) / S::TX, (a.g.ny + S::TY - 1) / S::TY, tile_x, tile_y)) return;
  fused_tile<S, FORM, MOMENTS, BC, false>(s, a, m, tile_x, tile_y);
}

template <class S, int BC>
__global__ __launch_bounds__(S::NT) void k_phi(const float* __restrict__ snew, const double* phi_in, double* phi_out,
                                                Grid g) {
  int tx, ty;
  if (!xcd_tile((g.nx + S::TX - 1) / S::TX, (g.ny + S::TY - 1) / S::TY, tx, ty)) return;
  phi_tile<S, BC>(snew, phi_in, phi_out, g, tx, ty);
}

// Initial state, pass 1: node-local f^eq(P = 0, rho(phi0), u0) and
// h^eq(phi0, mu(phi0), u0) (Eqs. 31-32; reading A11) into the f and h planes
// of s_tmp; phi (FP64); (phi u) = phi0 u0 into s0.
__global__ __launch_bounds__(256) void k_init_local(const float* __restrict__ phi0, const float* __restrict__ ux0,
                                                    const float* __restrict__ uy0, float* __restrict__ s_tmp,
                                                    float* __restrict__ s0, double* __restrict__ phi, Grid g, Phys c) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= g.pitch || y >= g.ny) return;
  const size_t on = nbase(g, x, y);
  if (x >= g.nx) {
    // lanes past nx in the last 64-node segment of a row: no step writes
    // them, so they are zeroed here (equal states then save to equal blobs)
    for (int k = 0; k < kNPL; ++k) {
      s_tmp[on + (unsigned)(k * 64)] = 0.0f;
      s0[on + (unsigned)(k * 64)] = 0.0f;
    }
    phi[(long long)y * g.pitch + x] = 0.0;
    return;
  }
  const double p0 = (double)phi0[(long long)y * g.nx + x];
  double sl = 0.0;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const int sx = wrap_or_reflect(x + cx(i), g.nx, c.wall_x), sy = wrap_or_reflect(y + cy(i), g.ny, c.wall_y);
    sl += wtd(i) * ((double)phi0[(long long)sy * g.nx + sx] - p0);
  }
  const float lap = (float)(6.0 * sl);
  const float mu = c.beta4 * (float)p0 * (float)((p0 - 1.0) * (p0 + 1.0)) - c.kappa * lap;
  const float ux = ux0 ? ux0[(long long)y * g.nx + x] : 0.f;
  const float uy = uy0 ? uy0[(long long)y * g.nx + x] : 0.f;
  const float rho = rho_of(p0, c);
  const float usq = ux * ux + uy * uy;
  const float etamu = c.eta * mu;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float cu = (float)cx(i) * ux + (float)cy(i) * uy;
    const float si = 3.0f * cu + 4.5f * cu * cu - 1.5f * usq;
    s_tmp[on + (unsigned)((kPF + i) * 64)] = wt(i) * CS2 * rho * si;
    s_tmp[on + (unsigned)((kPH + i) * 64)] = (i == 0) ? 0.0f : wt(i) * etamu + wt(i) * (float)p0 * 3.0f * cu;
  }
  phi[(long long)y * g.pitch + x] = p0;
  s0[on + (unsigned)(kPJ * 64)] = (float)p0 * ux;
  s0[on + (unsigned)((kPJ + 1) * 64)] = (float)p0 * uy;
}

// Initial state, pass 2: place node-local populations in the stored (post-
// collision) layout so that the pull of the first step returns them:
// slot j at y holds the value of node y + c_j, or the opp(j) value of y itself
// when y + c_j lies beyond a wall.  Slot 0 of h holds d0 = 0.
__global__ __launch_bounds__(256) void k_init_unstream(const float* __restrict__ s_tmp, float* __restrict__ s0, Grid g,
                                                       int wx, int wy) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= g.nx || y >= g.ny) return;
  const size_t on = nbase(g, x, y);
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    // the node that pulls this slot at the first step, and in which direction
    // (the inverse of src_base: plain, specular at a free-slip wall, bounced)
    int tx = x + cx(j), ty = y + cy(j);
    bool out_x = false, out_y = false;
    if (wx) out_x = (tx < 0) | (tx >= g.nx); else tx = (tx + g.nx) % g.nx;
    if (wy) out_y = (ty < 0) | (ty >= g.ny); else ty = (ty + g.ny) % g.ny;
    size_t src;
    int slot;
    if (!out_x && !out_y) { src = nbase(g, tx, ty); slot = j; }
    else if (out_x && !out_y && g.slip_x) { src = nbase(g, x, ty); slot = mirror_x(j); }
    else if (out_y && !out_x && g.slip_y) { src = nbase(g, tx, y); slot = mirror_y(j); }
    else { src = on; slot = opp(j); }
    s0[on + (unsigned)((kPF + j) * 64)] = s_tmp[src + (unsigned)((kPF + slot) * 64)];
    s0[on + (unsigned)((kPH + j) * 64)] = (j == 0) ? 0.0f : s_tmp[src + (unsigned)((kPH + slot) * 64)];
  }
}

// Deterministic sum of the phi plane: per-block partial sums, then one block.
__global__ __launch_bounds__(256) void k_sum_partial(const double* __restrict__ phi, Grid g, double* partial) {
  __shared__ double red[256];
  double acc = 0.0;
  const long long n = (long long)g.nx * g.ny;
  for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
    const long long y = k / g.nx, x = k - y * g.nx;
    acc += phi[y * g.pitch + x];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_final(const double* __restrict__ partial, int n, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) acc += partial[k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// Up to three device copies and one zero fill in one launch (checkpoints):
// every byte count is a multiple of 4 and every pointer 4-byte aligned.
struct CopyJob {
  const unsigned* src[3];
  unsigned* dst[3];
  long long n[3];        // words
  long long nv[3];       // leading 16-byte groups (0 unless both ends are 16-byte aligned)
  unsigned* zero;        // words set to 0
  long long nzero;
};

// Each job: its 16-byte groups first, then the words past the last group.
__global__ __launch_bounds__(256) void k_copy_jobs(CopyJob j) {
  const long long stride = (long long)gridDim.x * 256, t0 = (long long)blockIdx.x * 256 + threadIdx.x;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const uint4* s4 = reinterpret_cast<const uint4*>(j.src[q]);
    uint4* d4 = reinterpret_cast<uint4*>(j.dst[q]);
    for (long long k = t0; k < j.nv[q]; k += stride) d4[k] = s4[k];
    for (long long k = 4 * j.nv[q] + t0; k < j.n[q]; k += stride) j.dst[q][k] = j.src[q][k];
  }
  for (long long k = t0; k < j.nzero; k += stride) j.zero[k] = 0u;
}

__global__ void k_fill_int(int* p, int v, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}


template <class S>
dim3 tile_grid(const Grid& g) {
  const int ntiles = ((g.nx + S::TX - 1) / S::TX) * ((g.ny + S::TY - 1) / S::TY);
  return dim3((ntiles + kXcds - 1) / kXcds * kXcds);
}

// A launch whose start and stop times events t0/t1 take from the dispatch
// itself when given (timed steps), else a plain launch.
#define PFLBM_LAUNCH(K, GRID, BLOCK, ST, T0, T1, ...)                         \
  do {                                                                        \
    if (T0) hipExtLaunchKernelGGL(K, GRID, BLOCK, 0, ST, T0, T1, 0, __VA_ARGS__); \
    else hipLaunchKernelGGL(K, GRID, BLOCK, 0, ST, __VA_ARGS__);              \
  } while (0)

template <class S, int FORM, int BC>
hipError_t launch_fused_t(const StepArgs& a, const MomentArgs& m, bool moments, hipStream_t st, hipEvent_t t0,
                          hipEvent_t t1) {
  if (moments) hipLaunchKernelGGL((k_fused<S, FORM, true, BC>), tile_grid<S>(a.g), dim3(S::NT), 0, st, a, m);
  else PFLBM_LAUNCH((k_fused<S, FORM, false, BC>), tile_grid<S>(a.g), dim3(S::NT), st, t0, t1, a, m);
  return hipGetLastError();
}

// Single lattices: every boundary set-up in shape 0; periodic lattices also
// in the other shapes (step only; the moments run in shape 0).
template <int FORM>
hipError_t launch_form(int shape, const StepArgs& a, const MomentArgs& m, bool moments, hipStream_t st, hipEvent_t t0,
                       hipEvent_t t1) {
  const int bc = a.c.wall_x | (a.c.wall_y << 1);
  if (!moments && bc == 0) {
    switch (shape) {
      case 1: return launch_fused_t<S1, FORM, 0>(a, m, false, st, t0, t1);
      case 2: return launch_fused_t<S2, FORM, 0>(a, m, false, st, t0, t1);
      case 3: return launch_fused_t<S3, FORM, 0>(a, m, false, st, t0, t1);
      default: break;
    }
  }
  switch (bc) {
    case 0: return launch_fused_t<S0, FORM, 0>(a, m, moments, st, t0, t1);
    case 1: return launch_fused_t<S0, FORM, 1>(a, m, moments, st, t0, t1);
    case 2: return launch_fused_t<S0, FORM, 2>(a, m, moments, st, t0, t1);
    default: return launch_fused_t<S0, FORM, 3>(a, m, moments, st, t0, t1);
  }
}

hipError_t dispatch(int form, int shape, const StepArgs& a, const MomentArgs& m, bool moments, hipStream_t st,
                    hipEvent_t t0, hipEvent_t t1) {
  switch (form) {
    case 0: return launch_form<0>(shape, a, m, moments, st, t0, t1);
    case 1: return launch_form<1>(shape, a, m, moments, st, t0, t1);
    case 2: return launch_form<2>(shape, a, m, moments, st, t0, t1);
    case 3: return launch_form<3>(shape, a, m, moments, st, t0, t1);
    case 4: return launch_form<4>(shape, a, m, moments, st, t0, t1);
    case 5: return launch_form<5>(shape, a, m, moments, st, t0, t1);
    case 6: return launch_form<6>(shape, a, m, moments, st, t0, t1);
    case 7: return launch_form<7>(shape, a, m, moments, st, t0, t1);
    default: return hipErrorInvalidValue;
  }
}

template <class S>
hipError_t launch_phi_t(const float* snew, const double* phi_in, double* phi_out, const Grid& g, int bc,
                        hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  switch (bc) {
    case 0: PFLBM_LAUNCH((k_phi<S, 0>), tile_grid<S>(g), dim3(S::NT), s, t0, t1, snew, phi_in, phi_out, g); break;
    case 1: PFLBM_LAUNCH((k_phi<S, 1>), tile_grid<S>(g), dim3(S::NT), s, t0, t1, snew, phi_in, phi_out, g); break;
    case 2: PFLBM_LAUNCH((k_phi<S, 2>), tile_grid<S>(g), dim3(S::NT), s, t0, t1, snew, phi_in, phi_out, g); break;
    default: PFLBM_LAUNCH((k_phi<S, 3>), tile_grid<S>(g), dim3(S::NT), s, t0, t1, snew, phi_in, phi_out, g); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fused(int form, int shape, const StepArgs& a, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  return dispatch(form, shape, a, MomentArgs{}, false, s, t0, t1);
}

hipError_t launch_moments(int form, const StepArgs& a, const MomentArgs& m, hipStream_t s) {
  return dispatch(form, 0, a, m, true, s, nullptr, nullptr);
}

hipError_t launch_phi(const float* snew, const double* phi_in, double* phi_out, const Grid& g, int wall_x, int wall_y,
                      int shape, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  const int bc = wall_x | (wall_y << 1);
  switch (shape) {
    case 1: return launch_phi_t<S1>(snew, phi_in, phi_out, g, bc, s, t0, t1);
    case 2: return launch_phi_t<S2>(snew, phi_in, phi_out, g, bc, s, t0, t1);
    case 3: return launch_phi_t<S3>(snew, phi_in, phi_out, g, bc, s, t0, t1);
    default: return launch_phi_t<S0>(snew, phi_in, phi_out, g, bc, s, t0, t1);
  }
}

hipError_t launch_init(const float* phi0, const float* ux0, const float* uy0, float* s_tmp, float* s0, double* phi,
                       const Grid& g, const Phys& c, hipStream_t s) {
  dim3 grid((g.nx + 63) / 64, (g.ny + 3) / 4);
  hipLaunchKernelGGL(k_init_local, grid, dim3(256), 0, s, phi0, ux0, uy0, s_tmp, s0, phi, g, c);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_init_unstream, grid, dim3(256), 0, s, s_tmp, s0, g, c.wall_x, c.wall_y);
  return hipGetLastError();
}

hipError_t launch_phi_sum(const double* phi, const Grid& g, double* partial, int npartial, double* out, hipStream_t s) {
  // no more partial sums than 256-node blocks (small lattices)
  const long long nb = ((long long)g.nx * g.ny + 255) / 256;
  if (nb < npartial) npartial = (int)nb;
  hipLaunchKernelGGL(k_sum_partial, dim3(npartial), dim3(256), 0, s, phi, g, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, partial, npartial, out);
  return hipGetLastError();
}

hipError_t launch_copies(const void* const* src, void* const* dst, const size_t* bytes, int njobs, void* zero,
                         size_t zero_bytes, hipStream_t s) {
  CopyJob j{};
  long long tot = 0;
  for (int k = 0; k < 3; ++k) {
    j.src[k] = k < njobs ? (const unsigned*)src[k] : nullptr;
    j.dst[k] = k < njobs ? (unsigned*)dst[k] : nullptr;
    j.n[k] = k < njobs ? (long long)(bytes[k] / 4) : 0;
    const bool al = (((uintptr_t)j.src[k] | (uintptr_t)j.dst[k]) & 15) == 0;
    j.nv[k] = al ? j.n[k] / 4 : 0;
    tot += j.n[k] - 3 * j.nv[k];   // work items: one per group, one per leftover word
  }
  j.zero = (unsigned*)zero;
  j.nzero = zero ? (long long)(zero_bytes / 4) : 0;
  tot += j.nzero;
  const long long want = (tot + 255) / 256;
  const unsigned blocks = (unsigned)(want < 8192 ? (want < 1 ? 1 : want) : 8192);
  hipLaunchKernelGGL(k_copy_jobs, dim3(blocks), dim3(256), 0, s, j);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int value, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, p, value, n);
  return hipGetLastError();
}

}  // namespace pflbm
