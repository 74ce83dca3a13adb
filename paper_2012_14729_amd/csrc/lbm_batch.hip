// Batched engine: its device kernels (persistent walks over a tile list of
// every instance) and the C-ABI host code (declarations in include/lbm.h).
//
// `count` independent periodic lattices share one caller-provided workspace:
//   [instance descriptors][tile list][status ints][rho0 sums][partial sums]
//   then, per instance, the same arrays as a single lattice (two interleaved
//   state arrays, FP64 phi).
// A step is launches over one tile list covering every instance (sorted by
// tile shape, then force form): per tile shape, the fused collide-stream
// kernel (one launch for every form, or one per form; persistent workgroups
// or one per tile), then per tile shape the order-parameter kernel (one
// workgroup per tile).  Steps are
// replayed from a HIP graph captured once per batch (buffer A -> B -> A ...),
// so the host issues one graph launch per kChunk steps.
//
// Launch shapes are chosen by timing: at creation every candidate (one
// kernel for all forms or one per form; interior addressing on or off;
// persistent workgroups per CU, or one workgroup per tile) runs a few steps
// on the batch itself, the fastest is kept, and the initial state is rebuilt.
// Choices are cached per batch signature for the process, and in the file
// named by PFLBM_TUNE_CACHE if set; PFLBM_BATCH_TUNE=0 skips the timing and
// PFLBM_BATCH_CFG=split,fast,blocks_per_cu forces a shape (diagnostics).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_tile.hpp"

// ---------------------------------------------------------------------------
// Device side: the batched step kernels over the tile list.
// ---------------------------------------------------------------------------
namespace pflbm {

// One tile of one instance, with everything the tile's first loads need (64
// bytes, one scalar load): the instance's buffers as byte offsets into the
// batch workspace (the kernels rebuild the pointers from the workspace base,
// a kernel argument, so that they are known to address global memory) and
// its grid.  The force form and constants come from the instance's Phys
// entry, which is needed only after the order parameter has been staged.
struct TileJob {
  long long off_s[2];   // population buffers 0 and 1
  long long off_phi;    // order parameter
  int inst, form, tx, ty;
  int nx, ny, pitch, rowe;
  int fast, pad;
};
static_assert(sizeof(TileJob) == 64, "one 64-byte scalar load per tile");

namespace {

// Batched step: persistent workgroups walk a tile list covering every
// instance (sorted by force form, then instance).  A launch covers the tile
// range [t0, t1), cut into 8 contiguous bands, one per XCD; the workgroups of
// an XCD stride through its band, so consecutive tiles of an instance share
// that XCD's L2.
__device__ __forceinline__ void band(int t0, int t1, int& first, int& end, int& stride) {
  const int per = (t1 - t0 + kXcds - 1) / kXcds;
  const int beg = t0 + (int)(blockIdx.x % kXcds) * per;
  end = min(t1, beg + per);
  first = beg + (int)(blockIdx.x / kXcds);
  stride = (int)(gridDim.x / kXcds);
}

// Addressing paths of a batched step kernel: every tile general (0);
// interior tiles on the interior path, the others general (1); every tile
// wrapped (2, when every instance's arrays allow it).  One kernel holds at
// most two paths: the compiler merges the bodies of a kernel into shared
// blocks, and a kernel with the interior and the wrapped body measured no
// faster than either path alone.
constexpr int kBatchGeneral = 0, kBatchInterior = 1, kBatchWrapped = 2;

template <class S, int FORM, int PATHS>
__device__ __forceinline__ void batch_tile(Lds<S>& s, const StepArgs& a, int tx, int ty) {
  if constexpr (PATHS == kBatchInterior) fused_tile<S, FORM, false, 0, true>(s, a, MomentArgs{}, tx, ty);
  else if constexpr (PATHS == kBatchWrapped) tile_impl<S, FORM, false, 0, kPathWrapped, true>(s, a, MomentArgs{}, tx, ty);
  else tile_impl<S, FORM, false, 0, kPathGeneral, true>(s, a, MomentArgs{}, tx, ty);
}

// Step arguments of a tile with its pointers rebuilt from the workspace base,
// a kernel argument: pointers read from memory would be generic, and every
// access through them a flat one (which also counts against the LDS wait
// counter).
__device__ __forceinline__ StepArgs batch_args(const TileJob& j, const Phys* phys, int* status, int parity, char* ws) {
  StepArgs a;
  // a conditional, not j.off_s[parity]: a run-time index into the local
  // copy would place it in private memory
  a.sin = (const float*)(ws + (parity ? j.off_s[1] : j.off_s[0]));
  a.sout = (float*)(ws + (parity ? j.off_s[0] : j.off_s[1]));
  a.phi = (const double*)(ws + j.off_phi);
  a.status = status + j.inst;
  a.g.nx = j.nx;
  a.g.ny = j.ny;
  a.g.pitch = j.pitch;
  a.g.ncx = j.pitch >> 6;
  a.g.ps = (long long)j.pitch * j.ny;
  a.g.rowe = j.rowe;
  a.g.fast = j.fast;
  a.g.slip_x = a.g.slip_y = 0;   // periodic instances
  a.c = phys[j.inst];
  return a;
}

// FORM >= 0: every tile of [t0, t1) has that force form (the tile list is
// sorted by form); FORM < 0: any form, dispatched per tile.
template <class S, int FORM, int PATHS>
__global__ __launch_bounds__(S::NT) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_fused(
    const TileJob* __restrict__ jobs, const Phys* __restrict__ phys, int* status, char* ws, int t0, int t1,
    int parity) {
  __shared__ Lds<S> s;
  int first, end, stride;
  band(t0, t1, first, end, stride);
  for (int t = first; t < end; t += stride) {
    const TileJob tr = jobs[t];
    __syncthreads();   // the previous tile is done with the LDS
    const StepArgs a = batch_args(tr, phys, status, parity, ws);
    if constexpr (FORM >= 0) {
      batch_tile<S, FORM, PATHS>(s, a, tr.tx, tr.ty);
    } else {
      switch (tr.form) {
        case 0: batch_tile<S, 0, PATHS>(s, a, tr.tx, tr.ty); break;
        case 1: batch_tile<S, 1, PATHS>(s, a, tr.tx, tr.ty); break;
        case 2: batch_tile<S, 2, PATHS>(s, a, tr.tx, tr.ty); break;
        case 3: batch_tile<S, 3, PATHS>(s, a, tr.tx, tr.ty); break;
        case 4: batch_tile<S, 4, PATHS>(s, a, tr.tx, tr.ty); break;
        case 5: batch_tile<S, 5, PATHS>(s, a, tr.tx, tr.ty); break;
        case 6: batch_tile<S, 6, PATHS>(s, a, tr.tx, tr.ty); break;
        default: batch_tile<S, 7, PATHS>(s, a, tr.tx, tr.ty); break;
      }
    }
  }
}

// The order-parameter pass needs only the tile's own entry (no constants).
template <class S>
__global__ __launch_bounds__(S::NT) void k_batch_phi(const TileJob* __restrict__ jobs, char* ws, int t0, int t1,
                                                     int parity) {
  int first, end, stride;
  band(t0, t1, first, end, stride);
  for (int t = first; t < end; t += stride) {
    const TileJob j = jobs[t];
    Grid g;
    g.nx = j.nx;
    g.ny = j.ny;
    g.pitch = j.pitch;
    g.ncx = j.pitch >> 6;
    g.ps = (long long)j.pitch * j.ny;
    g.rowe = j.rowe;
    g.fast = j.fast;
    g.slip_x = g.slip_y = 0;
    double* phi = (double*)(ws + j.off_phi);
    phi_tile<S, 0, true>((const float*)(ws + (parity ? j.off_s[0] : j.off_s[1])), phi, phi, g, j.tx, j.ty);
  }
}

}  // namespace

}  // namespace pflbm

namespace pflbm {

template <class S, int FORM>
void launch_batch_form(int paths, dim3 grid, hipStream_t s, const TileJob* jobs, const Phys* phys, int* status,
                       char* ws, int t0, int t1, int parity) {
  if (paths == kBatchInterior)
    hipLaunchKernelGGL((k_batch_fused<S, FORM, kBatchInterior>), grid, dim3(S::NT), 0, s, jobs, phys, status, ws, t0,
                       t1, parity);
  else if (paths == kBatchWrapped)
    hipLaunchKernelGGL((k_batch_fused<S, FORM, kBatchWrapped>), grid, dim3(S::NT), 0, s, jobs, phys, status, ws, t0,
                       t1, parity);
  else
    hipLaunchKernelGGL((k_batch_fused<S, FORM, kBatchGeneral>), grid, dim3(S::NT), 0, s, jobs, phys, status, ws, t0,
                       t1, parity);
}

template <class S>
void launch_batch_shape(int form, int fast, dim3 grid, hipStream_t s, const TileJob* jobs, const Phys* phys,
                        int* status, char* ws, int t0, int t1, int parity) {
  switch (form) {
    case 0: launch_batch_form<S, 0>(fast, grid, s, jobs, phys, status, ws, t0, t1, parity); break;
    case 1: launch_batch_form<S, 1>(fast, grid, s, jobs, phys, status, ws, t0, t1, parity); break;
    case 2: launch_batch_form<S, 2>(fast, grid, s, jobs, phys, status, ws, t0, t1, parity); break;
    case 3: launch_batch_form<S, 3>(fast, grid, s, jobs, phys, status, ws, t0, t1, parity); break;
    case 4: launch_batch_form<S, 4>(fast, grid, s, jobs, phys, status, ws, t0, t1, parity); break;
    case 5: launch_batch_form<S, 5>(fast, grid, s, jobs, phys, status, ws, t0, t1, parity); break;
    case 6: launch_batch_form<S, 6>(fast, grid, s, jobs, phys, status, ws, t0, t1, parity); break;
    case 7: launch_batch_form<S, 7>(fast, grid, s, jobs, phys, status, ws, t0, t1, parity); break;
    default: launch_batch_form<S, -1>(fast, grid, s, jobs, phys, status, ws, t0, t1, parity); break;
  }
}

// Persistent batched step kernels over the tile range [t0, t1) of the tile
// list (periodic instances); form < 0: one kernel for every form, else the
// tiles all have that form.
hipError_t launch_batch_fused(const TileJob* jobs, const Phys* phys, int* status, char* ws, int t0, int t1, int form,
                              int fast, int parity, int nblocks, int shape, hipStream_t s) {
  const dim3 grid(nblocks);
  switch (shape) {
    case 1: launch_batch_shape<S1>(form, fast, grid, s, jobs, phys, status, ws, t0, t1, parity); break;
    case 2: launch_batch_shape<S2>(form, fast, grid, s, jobs, phys, status, ws, t0, t1, parity); break;
    case 3: launch_batch_shape<S3>(form, fast, grid, s, jobs, phys, status, ws, t0, t1, parity); break;
    default: launch_batch_shape<S0>(form, fast, grid, s, jobs, phys, status, ws, t0, t1, parity); break;
  }
  return hipGetLastError();
}

hipError_t launch_batch_phi(const TileJob* jobs, char* ws, int t0, int t1, int parity, int nblocks, int shape,
                            hipStream_t s) {
  switch (shape) {
    case 1: hipLaunchKernelGGL(k_batch_phi<S1>, dim3(nblocks), dim3(S1::NT), 0, s, jobs, ws, t0, t1, parity); break;
    case 2: hipLaunchKernelGGL(k_batch_phi<S2>, dim3(nblocks), dim3(S2::NT), 0, s, jobs, ws, t0, t1, parity); break;
    case 3: hipLaunchKernelGGL(k_batch_phi<S3>, dim3(nblocks), dim3(S3::NT), 0, s, jobs, ws, t0, t1, parity); break;
    default: hipLaunchKernelGGL(k_batch_phi<S0>, dim3(nblocks), dim3(S0::NT), 0, s, jobs, ws, t0, t1, parity); break;
  }
  return hipGetLastError();
}

// Resident workgroups per CU of the batched step kernel of a tile shape (the
// any-form kernel with the interior path, the largest register footprint).
int fused_blocks_per_cu(int shape) {
  int n = 0;
  hipError_t e;
  switch (shape) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_fused<S1, -1, kBatchInterior>, S1::NT, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_fused<S2, -1, kBatchInterior>, S2::NT, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_fused<S3, -1, kBatchInterior>, S3::NT, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_fused<S0, -1, kBatchInterior>, S0::NT, 0); break;
  }
  return (e != hipSuccess || n < 1) ? 1 : n;
}

}  // namespace pflbm

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
using namespace pflbm;

namespace {

template <typename... A>
int bfail(int code, const char* fmt, A... args) {
  return set_error(code, fmt, args...);
}

#define BHIP(expr)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return bfail(LBM_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kPartials = 512;      // same reduction shape as a single lattice
constexpr int kChunk = 16;          // steps per graph replay (even)
size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct InstLayout {
  Grid g;
  size_t s[2], phi;
};

struct BatchLayout {
  size_t desc, tiles, status, sums, partial, total;
  std::vector<InstLayout> inst;
  int ntiles;
};

// Tile-shape policies: 0..kNumShapes-1 give every instance that shape;
// kPolicyFit gives an instance 32x8 tiles where 64-wide ones would leave
// more lanes of its last tile column idle, else 64x8 (sides that are not a
// multiple of 64; measured on 32..512-node instances: 6-7 % faster steps
// for the instances up to 320 nodes wide).
constexpr int kPolicyFit = kNumShapes;

// Launch shape of the batched step.
struct BatchCfg {
  int split;    // 1: one fused launch per force form and tile shape; 0: one launch per tile shape
  int fast;     // addressing paths: kBatchGeneral, kBatchInterior or kBatchWrapped
  int bpc;      // persistent workgroups per CU; 0: one workgroup per tile
  int policy;   // tile-shape policy
  double ms;    // measured time per step (ms), 0 if not timed
};

int tiles_x(int nx, int shape) { return (nx + kShapeTX[shape] - 1) / kShapeTX[shape]; }
int tiles_y(int ny, int shape) { return (ny + kShapeTY[shape] - 1) / kShapeTY[shape]; }
int ntiles_of(int nx, int ny, int shape) { return tiles_x(nx, shape) * tiles_y(ny, shape); }

int shape_for(int nx, int policy) {
  if (policy < kNumShapes) return policy;
  const int idle64 = tiles_x(nx, 0) * kShapeTX[0] - nx, idle32 = tiles_x(nx, 2) * kShapeTX[2] - nx;
  return idle32 < idle64 ? 2 : 0;
}

// Room for the tile list of any policy: each instance's most tiles.
BatchLayout layout(const lbm_params* p, int count) {
  BatchLayout L{};
  L.ntiles = 0;
  for (int k = 0; k < count; ++k) {
    int n = 0;
    for (int sh = 0; sh < kNumShapes; ++sh) n = std::max(n, ntiles_of(p[k].nx, p[k].ny, sh));
    L.ntiles += n;
  }
  size_t o = 0;
  L.desc = o; o = up(o + sizeof(Phys) * (size_t)count);
  L.tiles = o; o = up(o + sizeof(TileJob) * (size_t)L.ntiles);
  L.status = o; o = up(o + sizeof(int) * (size_t)count);
  L.sums = o; o = up(o + sizeof(double) * (size_t)count);
  L.partial = o; o = up(o + sizeof(double) * kPartials * (size_t)count);
  L.inst.resize(count);
  for (int k = 0; k < count; ++k) {
    InstLayout& I = L.inst[k];
    I.g.nx = p[k].nx;
    I.g.ny = p[k].ny;
    I.g.pitch = (p[k].nx + 63) / 64 * 64;   // as a single lattice, so results match bit for bit
    I.g.ncx = I.g.pitch / 64;
    I.g.ps = (long long)I.g.pitch * p[k].ny;
    I.g.rowe = I.g.ncx * kSegE;
    I.g.fast = fast_bits(I.g.ps);
    if (const char* e = std::getenv("PFLBM_GENERAL_PATH")) {
      if (e[0] == '1') I.g.fast = 0;
      if (e[0] == '2') I.g.fast &= kFastInterior;
    }
    const size_t sbytes = (size_t)kNPL * (size_t)I.g.ps * sizeof(float);
    for (int b = 0; b < 2; ++b) { I.s[b] = o; o = up(o + sbytes); }
    I.phi = o; o = up(o + (size_t)I.g.ps * sizeof(double));
  }
  L.total = o;
  return L;
}

int validate_one(const lbm_params* p, int k) {
  size_t dummy;
  const int r = lbm_workspace_bytes(p, &dummy);   // same rules as a single lattice
  if (r != LBM_OK) {
    char msg[400];
    snprintf(msg, sizeof(msg), "%s", lbm_last_error());
    return bfail(r, "instance %d: %s", k, msg);
  }
  if (p->wall_x || p->wall_y) return bfail(LBM_E_UNSUPPORTED, "instance %d: the batched engine is periodic only", k);
  return LBM_OK;
}

}  // namespace

// Host copy of an instance's step arguments for both ping-pong parities
// (a[p] reads population buffer p and writes buffer 1 - p), for the moments.
struct BatchInst {
  StepArgs a[2];
  long long off_s[2];
  long long off_phi, off_status;
  int form;
};

struct lbm_batch {
  int count;
  BatchLayout L;
  char* ws;
  std::vector<int> forms;
  std::vector<BatchInst> host;   // descriptors (as uploaded)
  int parity;                    // population buffer holding the current state
  int64_t step;
  int cus;                       // compute units of the device
  int forced_policy;             // PFLBM_BATCH_SHAPE, or -1
  bool wrap_ok;                  // every instance allows the wrapped addressing path
  int policy;                    // tile-shape policy of the uploaded tile list
  std::vector<int> ishape;       // tile shape of each instance under that policy
  int ntiles;                    // tiles of the list in use
  // tile list sorted by shape, then force form, then instance: the tiles of
  // shape sh and form f are [grp[sh][f], grp[sh][f + 1]), those of shape sh
  // [grp[sh][0], grp[sh][LBM_NUM_FORMS])
  int grp[kNumShapes][LBM_NUM_FORMS + 1];
  BatchCfg cfg;                  // launch shape in use
  hipStream_t cap;               // private stream used only for graph capture
  hipGraphExec_t exec;           // kChunk steps starting from parity 0
  Phys* d_phys() const { return (Phys*)(ws + L.desc); }
  TileJob* d_tiles() const { return (TileJob*)(ws + L.tiles); }
  int* d_status() const { return (int*)(ws + L.status); }
};

namespace {

// Workgroups of a launch over n tiles: a multiple of the 8 XCDs.
int grid_for(const lbm_batch* b, const BatchCfg& c, int n) {
  const int want = c.bpc > 0 ? b->cus * c.bpc : n;
  return std::max(8, (std::min(want, n) + 7) / 8 * 8);
}

// The step launches of the uploaded tile list (its policy is c.policy).
int launch_pair_steps(lbm_batch* b, const BatchCfg& c, int nsteps, int parity0, hipStream_t st) {
  int par = parity0;
  const BatchCfg one_per_tile{c.split, c.fast, 0, c.policy, 0.0};
  for (int n = 0; n < nsteps; ++n) {
    for (int sh = 0; sh < kNumShapes; ++sh) {
      const int* g = b->grp[sh];
      if (g[LBM_NUM_FORMS] == g[0]) continue;
      if (c.split) {
        for (int f = 0; f < LBM_NUM_FORMS; ++f)
          if (g[f + 1] > g[f])
            BHIP(launch_batch_fused(b->d_tiles(), b->d_phys(), b->d_status(), b->ws, g[f], g[f + 1], f, c.fast, par,
                                    grid_for(b, c, g[f + 1] - g[f]), sh, st));
      } else {
        BHIP(launch_batch_fused(b->d_tiles(), b->d_phys(), b->d_status(), b->ws, g[0], g[LBM_NUM_FORMS], -1, c.fast,
                                par, grid_for(b, c, g[LBM_NUM_FORMS] - g[0]), sh, st));
      }
    }
    // The order-parameter pass holds few registers: one workgroup per tile
    // keeps far more of them resident than the fused kernel's persistent grid.
    for (int sh = 0; sh < kNumShapes; ++sh) {
      const int* g = b->grp[sh];
      if (g[LBM_NUM_FORMS] > g[0])
        BHIP(launch_batch_phi(b->d_tiles(), b->ws, g[0], g[LBM_NUM_FORMS], par,
                              grid_for(b, one_per_tile, g[LBM_NUM_FORMS] - g[0]), sh, st));
    }
    par = 1 - par;
  }
  return LBM_OK;
}

// Sort the tiles of every instance by the shape `policy` gives it, then by
// force form, and upload the list (synchronises st).
int build_tiles(lbm_batch* b, int policy, hipStream_t st) {
  const int count = b->count;
  b->ishape.resize(count);
  for (int k = 0; k < count; ++k) b->ishape[k] = shape_for(b->L.inst[k].g.nx, policy);
  std::vector<int> order(count);
  for (int k = 0; k < count; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int i, int j) {
    return b->ishape[i] != b->ishape[j] ? b->ishape[i] < b->ishape[j] : b->forms[i] < b->forms[j];
  });
  std::vector<TileJob> tiles;
  tiles.reserve(b->L.ntiles);
  int k_at = 0;
  for (int sh = 0; sh < kNumShapes; ++sh)
    for (int f = 0; f <= LBM_NUM_FORMS; ++f) {
      // first tile of (sh, f): append the instances of this group
      b->grp[sh][f] = (int)tiles.size();
      if (f == LBM_NUM_FORMS) break;
      for (; k_at < count && b->ishape[order[k_at]] == sh && b->forms[order[k_at]] == f; ++k_at) {
        const int k = order[k_at];
        const InstLayout& I = b->L.inst[k];
        const int ntx = tiles_x(I.g.nx, sh), nty = tiles_y(I.g.ny, sh);
        for (int ty = 0; ty < nty; ++ty)
          for (int tx = 0; tx < ntx; ++tx) {
            TileJob j{};
            j.off_s[0] = (long long)I.s[0];
            j.off_s[1] = (long long)I.s[1];
            j.off_phi = (long long)I.phi;
            j.inst = k;
            j.form = f;
            j.tx = tx;
            j.ty = ty;
            j.nx = I.g.nx;
            j.ny = I.g.ny;
            j.pitch = I.g.pitch;
            j.rowe = I.g.rowe;
            j.fast = I.g.fast;
            tiles.push_back(j);
          }
      }
    }
  if (k_at != count || (int)tiles.size() > b->L.ntiles) return bfail(LBM_E_INVAL, "batch tile list: internal error");
  b->ntiles = (int)tiles.size();
  b->policy = policy;
  if (hipMemcpyAsync(b->ws + b->L.tiles, tiles.data(), sizeof(TileJob) * tiles.size(), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return bfail(LBM_E_HIP, "batch: uploading the tile list");
  return LBM_OK;
}

// Resident workgroups per CU of the fused kernel for the shapes in use.
int occupancy(const lbm_batch* b) {
  int occ = 64;
  for (int sh = 0; sh < kNumShapes; ++sh)
    if (b->grp[sh][LBM_NUM_FORMS] > b->grp[sh][0]) occ = std::min(occ, fused_blocks_per_cu(sh));
  return occ;
}

int build_graph(lbm_batch* b) {
  BHIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  BHIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  const int r = launch_pair_steps(b, b->cfg, kChunk, 0, b->cap);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap, &graph);
  if (r != LBM_OK) return r;
  if (e != hipSuccess) return bfail(LBM_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  const hipError_t e2 = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) return bfail(LBM_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
  return LBM_OK;
}

// Key of a batch for the tuning cache: device size, instance sizes, forms.
uint64_t signature(const lbm_params* p, const int32_t* forms, int count, int cus, int forced_policy, bool wrap_ok) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
  mix((uint64_t)cus);
  mix((uint64_t)(forced_policy + 1));
  mix((uint64_t)wrap_ok);
  mix((uint64_t)count);
  for (int k = 0; k < count; ++k) {
    mix((uint64_t)p[k].nx);
    mix((uint64_t)p[k].ny);
    mix((uint64_t)forms[k]);
  }
  return h;
}

std::mutex g_tune_mu;
std::map<uint64_t, BatchCfg> g_tune;
bool g_tune_file_read = false;

const char* tune_file() { return std::getenv("PFLBM_TUNE_CACHE"); }

void read_tune_file() {   // g_tune_mu held
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char* path = tune_file();
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  unsigned long long key;
  BatchCfg c{};
  while (fscanf(f, "%llx %d %d %d %d %lf", &key, &c.split, &c.fast, &c.bpc, &c.policy, &c.ms) == 6)
    g_tune[(uint64_t)key] = c;
  fclose(f);
}

void append_tune_file(uint64_t key, const BatchCfg& c) {   // g_tune_mu held
  const char* path = tune_file();
  if (!path) return;
  if (FILE* f = fopen(path, "a")) {
    fprintf(f, "%016llx %d %d %d %d %.6f\n", (unsigned long long)key, c.split, c.fast, c.bpc, c.policy, c.ms);
    fclose(f);
  }
}

// Average time per step of configuration c (2 untimed steps, then 4).
int time_cfg(lbm_batch* b, const BatchCfg& c, hipStream_t st, double* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BHIP(hipEventCreate(&e0));
  const hipError_t ec = hipEventCreate(&e1);
  int r = ec == hipSuccess ? LBM_OK : bfail(LBM_E_HIP, "hipEventCreate: %s", hipGetErrorString(ec));
  if (r == LBM_OK) r = launch_pair_steps(b, c, 2, 0, st);
  if (r == LBM_OK && hipEventRecord(e0, st) != hipSuccess) r = bfail(LBM_E_HIP, "hipEventRecord failed");
  if (r == LBM_OK) r = launch_pair_steps(b, c, 4, 0, st);
  if (r == LBM_OK && hipEventRecord(e1, st) != hipSuccess) r = bfail(LBM_E_HIP, "hipEventRecord failed");
  float t = 0.f;
  if (r == LBM_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess))
    r = bfail(LBM_E_HIP, "timing the batched step failed");
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  *ms = t / 4.0;
  return r;
}

// Initial states (Eqs. 31-32, reading A11) of every instance and clear flags.
int init_states(lbm_batch* b, const lbm_params* params, const float* const* d_phi0, hipStream_t st, bool sums) {
  char* ws = b->ws;
  for (int k = 0; k < b->count; ++k) {
    const InstLayout& I = b->L.inst[k];
    const Phys c0 = derive_phys(&params[k], 0.0);
    hipError_t e = launch_init(d_phi0[k], nullptr, nullptr, (float*)(ws + I.s[1]), (float*)(ws + I.s[0]),
                               (double*)(ws + I.phi), I.g, c0, st);
    if (e == hipSuccess && sums)   // sums of phi0 for rho0 (A12)
      e = launch_phi_sum((double*)(ws + I.phi), I.g, (double*)(ws + b->L.partial) + (size_t)k * kPartials, kPartials,
                         (double*)(ws + b->L.sums) + k, st);
    if (e != hipSuccess) return bfail(LBM_E_HIP, "batch init: %s", hipGetErrorString(e));
  }
  if (launch_fill_int(b->d_status(), 0, b->count, st) != hipSuccess) return bfail(LBM_E_HIP, "status fill");
  return LBM_OK;
}

// Pick the launch shape: cached, default, or the fastest candidate measured
// on this batch (the timing steps change the state; it is rebuilt after).
int choose_cfg(lbm_batch* b, const lbm_params* params, const int32_t* forms, const float* const* d_phi0,
               hipStream_t st) {
  const int policy0 = b->forced_policy >= 0 ? b->forced_policy : 0;
  const BatchCfg dflt{1, b->wrap_ok ? kBatchWrapped : kBatchInterior, 0, policy0, 0.0};
  if (const char* fc = std::getenv("PFLBM_BATCH_CFG")) {   // forced shape "split,paths,blocks_per_cu"
    BatchCfg c{0, 0, 0, policy0, 0.0};
    if (sscanf(fc, "%d,%d,%d", &c.split, &c.fast, &c.bpc) != 3 || c.split < 0 || c.split > 1 || c.fast < 0 ||
        c.fast > 2 || c.bpc < 0 || c.bpc > 64)
      return bfail(LBM_E_INVAL, "PFLBM_BATCH_CFG must be split,paths,blocks_per_cu (0/1, 0..2, 0..64)");
    if (c.fast == kBatchWrapped && !b->wrap_ok)
      return bfail(LBM_E_INVAL, "PFLBM_BATCH_CFG: the wrapped path needs every instance's arrays within 4 GiB");
    b->cfg = c;
    return build_tiles(b, c.policy, st);
  }
  const char* tv = std::getenv("PFLBM_BATCH_TUNE");
  if (tv && tv[0] == '0') {
    b->cfg = dflt;
    return build_tiles(b, dflt.policy, st);
  }
  const uint64_t key = signature(params, forms, b->count, b->cus, b->forced_policy, b->wrap_ok);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    read_tune_file();
    auto it = g_tune.find(key);
    const bool usable = it != g_tune.end() && (it->second.fast != kBatchWrapped || b->wrap_ok) &&
                        it->second.policy >= 0 && it->second.policy <= kPolicyFit &&
                        (b->forced_policy < 0 || it->second.policy == b->forced_policy);
    if (usable) {
      b->cfg = it->second;
      return build_tiles(b, b->cfg.policy, st);
    }
  }
  BatchCfg best = dflt;
  best.ms = 1e300;
  std::vector<int> policies;
  if (b->forced_policy >= 0) policies = {b->forced_policy};
  else policies = {0, 2, kPolicyFit};
  std::vector<std::vector<int>> seen;
  for (int pol : policies) {
    if (int r = build_tiles(b, pol, st)) return r;
    if (std::find(seen.begin(), seen.end(), b->ishape) != seen.end()) continue;   // same tiles as a policy timed
    seen.push_back(b->ishape);
    const int occ = occupancy(b);
    for (int split = 0; split <= 1; ++split)
      for (int fast = 0; fast <= (b->wrap_ok ? 2 : 1); ++fast)
        for (int bpc : {1, 2, 0}) {
          if (bpc > occ) continue;
          BatchCfg c{split, fast, bpc, pol, 0.0};
          double ms = 0.0;
          if (int r = time_cfg(b, c, st, &ms)) return r;
          if (ms < best.ms) {
            best = c;
            best.ms = ms;
          }
        }
  }
  if (b->policy != best.policy)
    if (int r = build_tiles(b, best.policy, st)) return r;
  if (int r = init_states(b, params, d_phi0, st, false)) return r;
  b->cfg = best;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = best;
  append_tune_file(key, best);
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_batch_workspace_bytes(const lbm_params* params, int32_t count, size_t* bytes) {
  if (!params || count <= 0 || !bytes) return bfail(LBM_E_INVAL, "bad arguments");
  for (int k = 0; k < count; ++k)
    if (int r = validate_one(&params[k], k)) return r;
  *bytes = layout(params, count).total;
  return LBM_OK;
}

int lbm_batch_create(lbm_batch** out, const lbm_params* params, const int32_t* forms, int32_t count, void* d_ws,
                     size_t ws_bytes, const float* const* d_phi0, void* stream) {
  if (!out) return bfail(LBM_E_INVAL, "batch is NULL");
  *out = nullptr;
  if (!params || !forms || count <= 0 || !d_phi0) return bfail(LBM_E_INVAL, "bad arguments");
  for (int k = 0; k < count; ++k) {
    if (int r = validate_one(&params[k], k)) return r;
    if (forms[k] < 0 || forms[k] >= LBM_NUM_FORMS) return bfail(LBM_E_INVAL, "instance %d: bad force form", k);
    if (!d_phi0[k]) return bfail(LBM_E_INVAL, "instance %d: phi0 is NULL", k);
  }
  if (!d_ws || ((uintptr_t)d_ws % kAlign) != 0) return bfail(LBM_E_INVAL, "workspace must be 256-byte aligned");
  BatchLayout L = layout(params, count);
  if (ws_bytes < L.total) return bfail(LBM_E_INVAL, "workspace too small: %zu < %zu", ws_bytes, L.total);
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return bfail(LBM_E_INVAL, "out of host memory");
  b->count = count;
  b->L = std::move(L);
  b->ws = (char*)d_ws;
  b->forms.assign(forms, forms + count);
  b->parity = 0;
  b->step = 0;
  b->cap = nullptr;
  b->exec = nullptr;
  b->forced_policy = -1;
  b->policy = -1;
  b->ntiles = 0;
  b->wrap_ok = true;
  for (int k = 0; k < count; ++k) b->wrap_ok = b->wrap_ok && (b->L.inst[k].g.fast & kFastWrap);
  if (const char* e = std::getenv("PFLBM_BATCH_SHAPE")) {   // diagnostics: force a tile-shape policy
    const int sh = atoi(e);
    if (sh < 0 || sh > kPolicyFit) {
      delete b;
      return bfail(LBM_E_INVAL, "PFLBM_BATCH_SHAPE must be 0..%d", kPolicyFit);
    }
    b->forced_policy = sh;
  }
  hipStream_t st = (hipStream_t)stream;
  auto cleanup = [&](int code) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return code;
  };
  char* ws = b->ws;
  if (int r = init_states(b, params, d_phi0, st, true)) return cleanup(r);
  std::vector<double> sums(count);
  if (hipMemcpyAsync(sums.data(), ws + b->L.sums, sizeof(double) * count, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return cleanup(bfail(LBM_E_HIP, "batch init: reading phi sums"));
  // descriptors for both parities
  b->host.resize(count);
  for (int k = 0; k < count; ++k) {
    const InstLayout& I = b->L.inst[k];
    const lbm_params& p = params[k];
    double rho0 = p.rho0;
    if (std::isnan(rho0)) {
      const double mphi = sums[k] / ((double)p.nx * p.ny);
      rho0 = p.rho1 * (1.0 + mphi) / 2.0 + p.rho2 * (1.0 - mphi) / 2.0;
    }
    const Phys c = derive_phys(&p, rho0);
    for (int par = 0; par < 2; ++par) {
      StepArgs& a = b->host[k].a[par];
      a.sin = (const float*)(ws + I.s[par]);
      a.sout = (float*)(ws + I.s[1 - par]);
      a.phi = (const double*)(ws + I.phi);
      a.status = b->d_status() + k;
      a.g = I.g;
      a.c = c;
    }
    b->host[k].off_s[0] = (long long)I.s[0];
    b->host[k].off_s[1] = (long long)I.s[1];
    b->host[k].off_phi = (long long)I.phi;
    b->host[k].off_status = (long long)((char*)(b->d_status() + k) - ws);
    b->host[k].form = forms[k];
  }
  std::vector<Phys> phys(count);
  for (int k = 0; k < count; ++k) phys[k] = b->host[k].a[0].c;
  if (hipMemcpyAsync(ws + b->L.desc, phys.data(), sizeof(Phys) * count, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return cleanup(bfail(LBM_E_HIP, "batch init: uploading descriptors"));
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess)
    return cleanup(bfail(LBM_E_HIP, "device query failed"));
  b->cus = cus;
  if (int r = choose_cfg(b, params, forms, d_phi0, st)) return cleanup(r);
  if (int r = build_graph(b)) return cleanup(r);
  *out = b;
  return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int32_t nsteps, void* stream) {
  if (!b) return bfail(LBM_E_INVAL, "batch is NULL");
  if (nsteps < 0) return bfail(LBM_E_INVAL, "nsteps must be >= 0");
  hipStream_t st = (hipStream_t)stream;
  int n = nsteps;
  if (b->parity == 1 && n > 0) {   // realign to the graph's starting buffer
    if (int r = launch_pair_steps(b, b->cfg, 1, 1, st)) return r;
    b->parity = 0;
    --n;
  }
  while (n >= kChunk) {
    BHIP(hipGraphLaunch(b->exec, st));
    n -= kChunk;
  }
  if (n > 0) {
    if (int r = launch_pair_steps(b, b->cfg, n, b->parity, st)) return r;
    b->parity = (b->parity + n) & 1;
  }
  b->step += nsteps;
  return LBM_OK;
}

int lbm_batch_moments(lbm_batch* b, int32_t k, float* d_phi, float* d_rho, float* d_ux, float* d_uy, float* d_p,
                      void* stream) {
  if (!b || k < 0 || k >= b->count) return bfail(LBM_E_INVAL, "bad batch or instance index");
  MomentArgs m{d_phi, d_rho, d_ux, d_uy, d_p, nullptr};
  BHIP(launch_moments(b->forms[k], b->host[k].a[b->parity], m, (hipStream_t)stream));
  return LBM_OK;
}

int lbm_batch_status(lbm_batch* b, int32_t* h_flags, void* stream) {
  if (!b || !h_flags) return bfail(LBM_E_INVAL, "NULL argument");
  std::vector<int> st(b->count);
  BHIP(hipMemcpyAsync(st.data(), b->d_status(), sizeof(int) * b->count, hipMemcpyDeviceToHost, (hipStream_t)stream));
  BHIP(hipStreamSynchronize((hipStream_t)stream));
  for (int k = 0; k < b->count; ++k) h_flags[k] = st[k] ? 1 : 0;
  return LBM_OK;
}

int lbm_batch_config(const lbm_batch* b, int32_t* split, int32_t* fast, int32_t* blocks_per_cu, double* ms_per_step) {
  if (!b || !split || !fast || !blocks_per_cu || !ms_per_step) return bfail(LBM_E_INVAL, "NULL argument");
  *split = b->cfg.split;
  *fast = b->cfg.fast;
  *blocks_per_cu = b->cfg.bpc;
  *ms_per_step = b->cfg.ms;
  return LBM_OK;
}

int lbm_batch_tile_shape(const lbm_batch* b, int32_t k, int32_t* tile_x, int32_t* tile_y) {
  if (!b || k < 0 || k >= b->count || !tile_x || !tile_y) return bfail(LBM_E_INVAL, "bad batch, instance or pointer");
  *tile_x = kShapeTX[b->ishape[k]];
  *tile_y = kShapeTY[b->ishape[k]];
  return LBM_OK;
}

int lbm_batch_destroy(lbm_batch* b) {
  if (!b) return LBM_OK;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return LBM_OK;
}

}  // extern "C"
