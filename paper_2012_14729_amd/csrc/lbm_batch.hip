// C-ABI host code of the batched engine (declarations in include/lbm.h).
//
// `count` independent periodic lattices share one caller-provided workspace:
//   [instance descriptors][tile list][status ints][rho0 sums][partial sums]
//   then, per instance, the same arrays as a single lattice (two interleaved
//   state arrays, FP64 phi).
// A step is two persistent launches over one tile list covering every
// instance (sorted by force form): the fused collide-stream kernel and the
// order-parameter kernel.  Steps are replayed from a HIP graph captured once
// per batch in pairs (buffer A -> B -> A), so the host issues one graph
// launch per kChunk steps.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.hpp"

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

int ntiles_of(const lbm_params& p) { return ((p.nx + kTX - 1) / kTX) * ((p.ny + kTY - 1) / kTY); }

BatchLayout layout(const lbm_params* p, int count) {
  BatchLayout L{};
  L.ntiles = 0;
  for (int k = 0; k < count; ++k) L.ntiles += ntiles_of(p[k]);
  size_t o = 0;
  L.desc = o; o = up(o + sizeof(BatchInst) * (size_t)count);
  L.tiles = o; o = up(o + sizeof(TileRef) * (size_t)L.ntiles);
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
    I.g.fast = 1;
    if (const char* e = std::getenv("PFLBM_GENERAL_PATH"))
      if (e[0] == '1') I.g.fast = 0;
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

struct lbm_batch {
  int count;
  BatchLayout L;
  char* ws;
  std::vector<int> forms;
  std::vector<BatchInst> host;   // descriptors (as uploaded)
  int parity;                    // population buffer holding the current state
  int64_t step;
  int nblocks;                   // persistent grid of the batched kernels
  hipStream_t cap;               // private stream used only for graph capture
  hipGraphExec_t exec;           // kChunk steps starting from parity 0
  BatchInst* d_inst() const { return (BatchInst*)(ws + L.desc); }
  TileRef* d_tiles() const { return (TileRef*)(ws + L.tiles); }
  int* d_status() const { return (int*)(ws + L.status); }
};

namespace {

int launch_pair_steps(lbm_batch* b, int nsteps, int parity0, hipStream_t st) {
  int par = parity0;
  for (int n = 0; n < nsteps; ++n) {
    BHIP(launch_batch_fused(b->d_inst(), b->d_tiles(), b->L.ntiles, par, b->nblocks, st));
    BHIP(launch_batch_phi(b->d_inst(), b->d_tiles(), b->L.ntiles, par, b->nblocks, st));
    par = 1 - par;
  }
  return LBM_OK;
}

int build_graph(lbm_batch* b) {
  BHIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  BHIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  const int r = launch_pair_steps(b, kChunk, 0, b->cap);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap, &graph);
  if (r != LBM_OK) return r;
  if (e != hipSuccess) return bfail(LBM_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  const hipError_t e2 = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) return bfail(LBM_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
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
  hipStream_t st = (hipStream_t)stream;
  auto cleanup = [&](int code) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return code;
  };
  char* ws = b->ws;
  // initial states (Eqs. 31-32, reading A11) and the sums of phi0 for rho0 (A12)
  for (int k = 0; k < count; ++k) {
    const InstLayout& I = b->L.inst[k];
    const Phys c0 = derive_phys(&params[k], 0.0);
    hipError_t e = launch_init(d_phi0[k], nullptr, nullptr, (float*)(ws + I.s[1]), (float*)(ws + I.s[0]),
                               (double*)(ws + I.phi), I.g, c0, st);
    if (e == hipSuccess)
      e = launch_phi_sum((double*)(ws + I.phi), I.g, (double*)(ws + b->L.partial) + (size_t)k * kPartials, kPartials,
                         (double*)(ws + b->L.sums) + k, st);
    if (e != hipSuccess) return cleanup(bfail(LBM_E_HIP, "batch init: %s", hipGetErrorString(e)));
  }
  if (launch_fill_int(b->d_status(), 0, count, st) != hipSuccess) return cleanup(bfail(LBM_E_HIP, "status fill"));
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
    b->host[k].form = forms[k];
  }
  // tile list: by force form, then instance, then row-major tiles
  std::vector<int> order(count);
  for (int k = 0; k < count; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int i, int j) { return forms[i] < forms[j]; });
  std::vector<TileRef> tiles;
  tiles.reserve(b->L.ntiles);
  for (int k : order) {
    const int ntx = (params[k].nx + kTX - 1) / kTX, nty = (params[k].ny + kTY - 1) / kTY;
    for (int ty = 0; ty < nty; ++ty)
      for (int tx = 0; tx < ntx; ++tx) tiles.push_back(TileRef{k, tx, ty, 0});
  }
  if (hipMemcpyAsync(ws + b->L.desc, b->host.data(), sizeof(BatchInst) * count, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(ws + b->L.tiles, tiles.data(), sizeof(TileRef) * tiles.size(), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return cleanup(bfail(LBM_E_HIP, "batch init: uploading descriptors"));
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess)
    return cleanup(bfail(LBM_E_HIP, "device query failed"));
  b->nblocks = std::max(8, cus * fused_blocks_per_cu() / 8 * 8);
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
    if (int r = launch_pair_steps(b, 1, 1, st)) return r;
    b->parity = 0;
    --n;
  }
  while (n >= kChunk) {
    BHIP(hipGraphLaunch(b->exec, st));
    n -= kChunk;
  }
  if (n > 0) {
    if (int r = launch_pair_steps(b, n, b->parity, st)) return r;
    b->parity = (b->parity + n) & 1;
  }
  b->step += nsteps;
  return LBM_OK;
}

int lbm_batch_moments(lbm_batch* b, int32_t k, float* d_phi, float* d_rho, float* d_ux, float* d_uy, float* d_p,
                      void* stream) {
  if (!b || k < 0 || k >= b->count) return bfail(LBM_E_INVAL, "bad batch or instance index");
  MomentArgs m{d_phi, d_rho, d_ux, d_uy, d_p};
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

int lbm_batch_destroy(lbm_batch* b) {
  if (!b) return LBM_OK;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return LBM_OK;
}

}  // extern "C"
