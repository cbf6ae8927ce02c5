// C ABI of the Euler hot-path library: topology planning, workspace layout,
// launch sequencing (per-block or batched, optionally as a hipGraph), the
// tile-shape autotuner and kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cfdhip.h"
#include "adjoint.h"
#include "viscous.h"
#include "cfd_internal.h"
#include "kernels.h"
#include "stage_kernel.h"

using namespace cfd;

namespace {

constexpr size_t ALIGN = 256;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
long long align_ll(long long x, long long a) { return (x + a - 1) / a * a; }

struct HBlock {
  int ni, nj, nk;
  std::vector<double> nodes;
};
struct HPatch {
  int block, face, lo[2], hi[2], kind;
  double params[MAXV];
  int param_index;
};
struct HConn {
  int a, fa, loa[2], hia[2], b, fb, lob[2], hib[2], orient;
};

struct EventPair {
  hipEvent_t a, b;
};

}  // namespace

struct cfd_ctx {
  cfd_config cfg{};
  int dim = 2, nvar = 4;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  int device = 0;
  std::string err;

  std::vector<HBlock> hblocks;
  std::vector<HPatch> hpatches;
  std::vector<HConn> hconns;
  bool finalized = false, bound = false, have_state = false, dt_valid = false;

  // planned tables (host copies of what is uploaded)
  std::vector<BlockDev> blocks;
  std::vector<TransferDev> xfers;
  std::vector<PatchDev> patches;
  std::vector<ChunkDev> chunks1, chunks2;     // phase 1 (pack + patches) and 2 (unpack), block-sorted
  std::vector<int> c1_begin, c2_begin;        // per-block chunk ranges (size nblocks + 1)
  std::vector<ChunkDev> chunksd;              // direct exchange: copies + patches, sorted by receiving block
  std::vector<int> cd_begin;                  // per-block ranges of chunksd (size nblocks + 1)
  std::vector<ChunkDev> chunksw;              // chunksd without the connections the stencil reads through
  std::vector<int> cw_begin;                  // per-block ranges of chunksw
  bool wrap_any = false;                      // some block axis is periodic onto itself
  int nvariants = 0;
  std::vector<std::vector<TileDev>> tiles_batched, tiles_block;  // per variant
  std::vector<std::vector<int>> tile_begin;                      // per variant, per block (+1)
  std::vector<long long> export_off;
  long long max_face_area = 0;
  bool need_bgather = true;  // some boundary cell is left to the boundary gather pass
  long long ncells = 0, nnodes = 0, max_cells = 0, max_padded = 0, max_pos = 0, padded_total = 0, max_faces = 0,
            max_nodes = 0;
  long long state_doubles = 0, metric_doubles = 0, xbuf_doubles = 0;
  bool has_farfield = false;
  int nparam = 0;  // parameter slots (inflow states, farfield states, stagnation or back pressures)

  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t off_rkD = 0, off_rkE = 0;  // classical RK4: stage input Y4 and Z = Q - dt/6 R(Y4)
  size_t off_stA = 0, off_stB = 0, off_stC = 0, off_metric = 0, off_nodes = 0, off_xbuf = 0, off_inflow = 0,
         off_dt = 0, off_dtmin = 0, off_err = 0, off_blocks = 0, off_xfers = 0, off_patches = 0, off_chunks1 = 0,
         off_chunks2 = 0, off_chunksd = 0, off_export = 0, off_chunksw = 0;
  std::vector<size_t> off_tiles_batched, off_tiles_block;

  // execution
  int variant = 0;
  int exec_mode = CFD_EXEC_BATCHED;
  int use_graph = 1;
  int ghost_mode = CFD_GHOSTS_DIRECT;
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  bool graph_valid = false;

  // adjoint
  bool adjoint = false;
  long long facebar_doubles = 0;
  size_t off_stD = 0, off_qbar = 0, off_facebar = 0, off_metricbar = 0, off_G = 0, off_T = 0, off_thetabar = 0,
         off_part = 0, off_partoff = 0, off_objchunks = 0, off_inflowlist = 0, off_walllist = 0,
         off_sumpart = 0, off_J = 0, off_facemap = 0, off_fmapoff = 0, off_vtiles = 0;
  std::vector<ChunkDev> obj_chunks;                  // objective, grouped by wall face
  std::vector<int> obj_begin;                        // per face (size 2*dim + 1)
  std::vector<int> facemap;                          // per block face position: donor transfer or -(patch+1)
  std::vector<long long> fmap_off;                   // [block * 6 + face]
  std::vector<TileDev> vtiles;                       // tiles of the fused 2D adjoint pass
  std::vector<long long> part_off;
  std::vector<int> inflow_list, wall_list;
  long long part_doubles = 0;
  static constexpr int SUM_PARTS = 1024;
  static constexpr int NORM_PARTS = 1024;
  size_t off_dtloc = 0, off_normpart = 0;
  bool viscous = false;   // laminar Navier-Stokes (cfg.viscosity > 0)
  long long center_doubles = 0;
  size_t off_centers = 0, off_npos = 0, off_rv = 0, off_vistiles = 0;
  std::vector<TileDev> vis_tiles;  // tiles of the fused 3D viscous pass
  bool freezing = false;  // workspace holds frozen-limiter arrays (cfd_enable_limiter_freezing)
  bool frozen = false;    // stage kernels use the frozen factors
  long long phi_doubles = 0;
  size_t off_phi = 0;

  // timing
  bool profiling = false;
  std::vector<EventPair> ev_pool;
  size_t ev_used = 0;
  double prof_ms = 0.0;
  long long prof_launches = 0;

  template <class T>
  T* dptr(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
  double* stA() const { return dptr<double>(off_stA); }
  double* stB() const { return dptr<double>(off_stB); }
  double* stC() const { return dptr<double>(off_stC); }
  double* metric() const { return dptr<double>(off_metric); }
};

namespace {

cfd_status fail(cfd_ctx* c, cfd_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return s;
}

#define HIP_TRY(ctx, expr)                                                                        \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) return fail(ctx, CFD_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int face_axis(int f) { return f >> 1; }

void face_extent(const HBlock& b, int dim, int face, int ext[2]) {
  int n[3] = {b.ni, b.nj, b.nk};
  int axis = face_axis(face);
  int m = 0;
  ext[0] = ext[1] = 1;
  for (int a = 0; a < dim; ++a)
    if (a != axis) ext[m++] = n[a];
}

Gas make_gas(double gamma) {
  Gas g;
  g.gamma = gamma;
  g.gm1 = gamma - 1.0;
  g.igm1 = 1.0 / (gamma - 1.0);
  g.g_gm1 = gamma / (gamma - 1.0);
  g.ig = 1.0 / gamma;
  g.ig2m1 = 1.0 / (gamma * gamma - 1.0);
  return g;
}

int inverse_orient(int o) {
  if (!(o & 4)) return o;
  return 4 | ((o & 2) ? 1 : 0) | ((o & 1) ? 2 : 0);
}

// workgroup w runs on XCD w % 8; give each XCD a contiguous run of spatially
// ordered tiles so halo re-reads of neighbouring tiles hit the same L2.
std::vector<TileDev> xcd_order(const std::vector<TileDev>& spatial, size_t begin, size_t end) {
  const size_t n = end - begin;
  std::vector<TileDev> out(n);
  const size_t q = n / 8, rem = n % 8;
  for (size_t w = 0; w < n; ++w) {
    const size_t x = w % 8, m = w / 8;
    const size_t start = x * q + std::min(x, rem);
    out[w] = spatial[begin + start + m];
  }
  return out;
}

cfd_status need(cfd_ctx* c, bool finalized, bool bound) {
  if (!c) return CFD_ERR_ARG;
  if (finalized && !c->finalized) return fail(c, CFD_ERR_STATE, "context is not finalized");
  if (bound && !c->bound) return fail(c, CFD_ERR_STATE, "no workspace bound");
  return CFD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Library-owned scratch for the entry point that allocates nothing
// (cfd_residual_norms_noalloc): the per-part partial sums of the residual
// norms.  One copy per GPU, alive until the process ends; its device address
// is looked up once per device (at cfd_create, with that device current) and
// only that address is passed to kernels.
constexpr int SCRATCH_DOUBLES = 1024 * 5;  // parts x variables, 40 KiB
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];
constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

static hipError_t scratch_setup(int device) {
  if (device < 0 || device >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_scratch_ptr[device] = static_cast<double*>(ptr);
  return e;
}

static double* scratch_of(int device) {
  if (device < 0 || device >= SCRATCH_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

extern "C" const char* cfd_version(void) { return "cfdhip 0.1 (gfx950, fp64)"; }

extern "C" const char* cfd_status_string(cfd_status s) {
  switch (s) {
    case CFD_OK: return "ok";
    case CFD_ERR_ARG: return "invalid argument";
    case CFD_ERR_STATE: return "call out of order";
    case CFD_ERR_TOPOLOGY: return "invalid topology";
    case CFD_ERR_GRID: return "invalid grid";
    case CFD_ERR_HIP: return "HIP runtime error";
    case CFD_ERR_NONFINITE: return "non-finite or non-physical state";
    case CFD_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

extern "C" const char* cfd_last_error(const cfd_ctx* c) { return c ? c->err.c_str() : ""; }

extern "C" cfd_status cfd_create(const cfd_config* cfg, void* stream, cfd_ctx** out) {
  if (!cfg || !out) return CFD_ERR_ARG;
  *out = nullptr;
  if (cfg->dim != 2 && cfg->dim != 3) return CFD_ERR_ARG;
  if (!(cfg->gamma > 1.0)) return CFD_ERR_ARG;
  if (cfg->limiter < CFD_LIM_NONE || cfg->limiter > CFD_LIM_VANALBADA) return CFD_ERR_ARG;
  if (cfg->flux < CFD_FLUX_ROE || cfg->flux > CFD_FLUX_STEGER_WARMING) return CFD_ERR_ARG;
  if (cfg->rk_stages < 1 || cfg->rk_stages > 8) return CFD_ERR_ARG;
  if (cfg->rk_scheme != CFD_RK_MSTAGE && cfg->rk_scheme != CFD_RK_CLASSIC4) return CFD_ERR_ARG;
  if (cfg->rk_scheme == CFD_RK_CLASSIC4 && cfg->rk_stages != 4) return CFD_ERR_ARG;
  if ((cfg->dt_mode == CFD_DT_CFL || cfg->dt_mode == CFD_DT_LOCAL) && !(cfg->cfl > 0.0)) return CFD_ERR_ARG;
  if (cfg->dt_mode == CFD_DT_FIXED && !(cfg->dt_fixed > 0.0)) return CFD_ERR_ARG;
  if (cfg->dt_mode != CFD_DT_CFL && cfg->dt_mode != CFD_DT_FIXED && cfg->dt_mode != CFD_DT_LOCAL)
    return CFD_ERR_ARG;
  if (!(cfg->efix >= 0.0) || !(cfg->muscl_eps >= 0.0)) return CFD_ERR_ARG;
  for (int v = 0; v < MAXV; ++v)
    if (!(cfg->lim_eps[v] >= 0.0)) return CFD_ERR_ARG;
  if (!(cfg->viscosity >= 0.0) || !std::isfinite(cfg->viscosity)) return CFD_ERR_ARG;
  if (cfg->viscosity > 0.0 && !(cfg->prandtl > 0.0)) return CFD_ERR_ARG;
  if (cfg->debug_flags & ~(CFD_CHECK_FINITE | CFD_NAN_GHOSTS)) return CFD_ERR_ARG;
  cfd_ctx* c = new cfd_ctx();
  c->cfg = *cfg;
  c->viscous = cfg->viscosity > 0.0;
  c->dim = cfg->dim;
  c->nvar = cfg->dim + 2;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  // Without a usable device the context still plans (add/set/connect/finalize);
  // binding a workspace then fails with CFD_ERR_HIP.
  if (hipGetDevice(&c->device) != hipSuccess) c->device = -1;
  // the no-allocation entry point's scratch: its address on this device
  // (failure is reported by that entry point, which cannot run without it)
  if (c->device >= 0) (void)scratch_setup(c->device);
  int n = 0;
  stage_variants(c->dim, &n);
  c->nvariants = n;
  *out = c;
  return CFD_OK;
}

static void release_graph(cfd_ctx* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
  c->graph_valid = false;
}

extern "C" cfd_status cfd_destroy(cfd_ctx* c) {
  if (!c) return CFD_ERR_ARG;
  release_graph(c);
  for (auto& e : c->ev_pool) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
  return CFD_OK;
}

extern "C" cfd_status cfd_add_block(cfd_ctx* c, int ni, int nj, int nk, const double* nodes, int* id) {
  if (!c || !nodes) return CFD_ERR_ARG;
  if (c->finalized) return fail(c, CFD_ERR_STATE, "add_block after finalize");
  if (c->dim == 2 && nk != 1) return fail(c, CFD_ERR_ARG, "2D blocks need nk = 1");
  if (ni < 2 || nj < 2 || (c->dim == 3 && nk < 2)) return fail(c, CFD_ERR_ARG, "block extents must be >= 2");
  if ((long long)ni * nj * nk > (1LL << 31)) return fail(c, CFD_ERR_ARG, "block too large");
  HBlock b{ni, nj, nk, {}};
  const size_t nn = (size_t)(ni + 1) * (nj + 1) * (c->dim == 3 ? nk + 1 : 1);
  b.nodes.assign(nodes, nodes + nn * c->dim);
  c->hblocks.push_back(std::move(b));
  if (id) *id = (int)c->hblocks.size() - 1;
  return CFD_OK;
}

static cfd_status check_range(cfd_ctx* c, int block, int face, const int lo[2], const int hi[2]) {
  if (block < 0 || block >= (int)c->hblocks.size()) return fail(c, CFD_ERR_ARG, "bad block id %d", block);
  if (face < 0 || face >= 2 * c->dim) return fail(c, CFD_ERR_ARG, "bad face %d", face);
  int ext[2];
  face_extent(c->hblocks[block], c->dim, face, ext);
  for (int t = 0; t < c->dim - 1; ++t)
    if (lo[t] < 0 || hi[t] > ext[t] || lo[t] >= hi[t])
      return fail(c, CFD_ERR_ARG, "range [%d,%d) outside face extent %d", lo[t], hi[t], ext[t]);
  return CFD_OK;
}

static bool has_params(int kind) {
  return kind != CFD_BC_SLIP_WALL && kind != CFD_BC_EXTRAP_OUTFLOW && kind != CFD_BC_NOSLIP_WALL;
}

// Checks the parameters of a patch kind and writes their stored form (MAXV
// doubles, the subsonic-inflow direction normalised) to out.
static cfd_status check_params(cfd_ctx* c, int kind, const double* params, double* out) {
  if (!params) return fail(c, CFD_ERR_ARG, "boundary kind %d needs parameters", kind);
  for (int v = 0; v < MAXV; ++v) out[v] = 0.0;
  const int nv = c->nvar, dim = c->dim;
  const int n = kind == CFD_BC_SUB_INFLOW ? 2 + dim : (kind == CFD_BC_SUB_OUTFLOW ? 1 : nv);
  for (int v = 0; v < n; ++v) {
    if (!std::isfinite(params[v])) return fail(c, CFD_ERR_NONFINITE, "boundary parameter %d is not finite", v);
    out[v] = params[v];
  }
  if (kind == CFD_BC_SUP_INFLOW || kind == CFD_BC_FARFIELD) {
    if (!(out[0] > 0.0) || !(out[nv - 1] > 0.0))
      return fail(c, CFD_ERR_NONFINITE, "boundary density and pressure must be positive");
  } else if (kind == CFD_BC_SUB_INFLOW) {
    if (!(out[0] > 0.0) || !(out[1] > 0.0))
      return fail(c, CFD_ERR_NONFINITE, "stagnation pressure and density must be positive");
    double s2 = 0.0;
    for (int d = 0; d < dim; ++d) s2 += out[2 + d] * out[2 + d];
    if (!(s2 > 0.0)) return fail(c, CFD_ERR_ARG, "subsonic inflow direction is zero");
    const double len = std::sqrt(s2);
    for (int d = 0; d < dim; ++d) out[2 + d] /= len;
  } else if (!(out[0] > 0.0)) {
    return fail(c, CFD_ERR_NONFINITE, "back pressure must be positive");
  }
  return CFD_OK;
}

extern "C" cfd_status cfd_set_bc(cfd_ctx* c, int block, int face, const int lo[2], const int hi[2], int kind,
                                 const double* params, int* patch_id) {
  if (!c || !lo || !hi) return CFD_ERR_ARG;
  if (c->finalized) return fail(c, CFD_ERR_STATE, "set_bc after finalize");
  cfd_status s = check_range(c, block, face, lo, hi);
  if (s != CFD_OK) return s;
  if (kind < CFD_BC_SLIP_WALL || kind > CFD_BC_NOSLIP_WALL) return fail(c, CFD_ERR_ARG, "bad boundary kind %d", kind);
  HPatch p{};
  p.block = block;
  p.face = face;
  p.kind = kind;
  p.param_index = -1;
  for (int t = 0; t < 2; ++t) {
    p.lo[t] = t < c->dim - 1 ? lo[t] : 0;
    p.hi[t] = t < c->dim - 1 ? hi[t] : 1;
  }
  if (has_params(kind)) {
    if ((s = check_params(c, kind, params, p.params)) != CFD_OK) return s;
    p.param_index = c->nparam++;
  }
  c->hpatches.push_back(p);
  if (patch_id) *patch_id = (int)c->hpatches.size() - 1;
  return CFD_OK;
}

extern "C" cfd_status cfd_connect(cfd_ctx* c, int a, int fa, const int loa[2], const int hia[2], int b, int fb,
                                  const int lob[2], const int hib[2], int orient) {
  if (!c || !loa || !hia || !lob || !hib) return CFD_ERR_ARG;
  if (c->finalized) return fail(c, CFD_ERR_STATE, "connect after finalize");
  cfd_status s = check_range(c, a, fa, loa, hia);
  if (s != CFD_OK) return s;
  s = check_range(c, b, fb, lob, hib);
  if (s != CFD_OK) return s;
  if (orient < 0 || orient > 7 || (c->dim == 2 && orient > 1)) return fail(c, CFD_ERR_ARG, "bad orient %d", orient);
  HConn h{};
  h.a = a;
  h.fa = fa;
  h.b = b;
  h.fb = fb;
  h.orient = orient;
  for (int t = 0; t < 2; ++t) {
    h.loa[t] = t < c->dim - 1 ? loa[t] : 0;
    h.hia[t] = t < c->dim - 1 ? hia[t] : 1;
    h.lob[t] = t < c->dim - 1 ? lob[t] : 0;
    h.hib[t] = t < c->dim - 1 ? hib[t] : 1;
  }
  int la0 = h.hia[0] - h.loa[0], la1 = h.hia[1] - h.loa[1];
  int lb0 = h.hib[0] - h.lob[0], lb1 = h.hib[1] - h.lob[1];
  bool ok = (orient & 4) ? (la0 == lb1 && la1 == lb0) : (la0 == lb0 && la1 == lb1);
  if (!ok) return fail(c, CFD_ERR_TOPOLOGY, "connection extents do not match under orient %d", orient);
  int na = face_axis(fa) == 0 ? c->hblocks[a].ni : (face_axis(fa) == 1 ? c->hblocks[a].nj : c->hblocks[a].nk);
  int nb = face_axis(fb) == 0 ? c->hblocks[b].ni : (face_axis(fb) == 1 ? c->hblocks[b].nj : c->hblocks[b].nk);
  if (na < NG || nb < NG) return fail(c, CFD_ERR_TOPOLOGY, "connected blocks need at least %d layers", NG);
  if (a == b && fa == fb) {
    // a face connected to itself must map every cell to a different one or it would copy onto itself
    bool overlap = !(h.hia[0] <= h.lob[0] || h.hib[0] <= h.loa[0]) && !(h.hia[1] <= h.lob[1] || h.hib[1] <= h.loa[1]);
    if (overlap && orient == 0) return fail(c, CFD_ERR_TOPOLOGY, "face connected onto itself");
  }
  c->hconns.push_back(h);
  return CFD_OK;
}

// ---------------------------------------------------------------------------

extern "C" cfd_status cfd_finalize(cfd_ctx* c, size_t* ws_bytes) {
  if (!c) return CFD_ERR_ARG;
  if (c->finalized) return fail(c, CFD_ERR_STATE, "already finalized");
  if (c->hblocks.empty()) return fail(c, CFD_ERR_STATE, "no blocks");
  if (c->adjoint && c->cfg.flux != CFD_FLUX_ROE)
    return fail(c, CFD_ERR_UNSUPPORTED, "the residual VJP is implemented for the Roe flux");
  if (c->adjoint && c->viscous)
    return fail(c, CFD_ERR_UNSUPPORTED, "the residual VJP is implemented for the Euler equations");
  if (c->adjoint && c->freezing)
    return fail(c, CFD_ERR_UNSUPPORTED, "the residual VJP differentiates the live limiter; freezing is not supported");
  if (c->adjoint)
    for (auto& p : c->hpatches)
      if (p.kind > CFD_BC_EXTRAP_OUTFLOW)
        return fail(c, CFD_ERR_UNSUPPORTED,
                    "the residual VJP covers slip-wall, supersonic-inflow and extrapolation patches");
  const int dim = c->dim, nv = c->nvar;
  const int nb = (int)c->hblocks.size();

  // --- boundary coverage: every boundary face cell exactly once -----------
  for (int b = 0; b < nb; ++b) {
    for (int f = 0; f < 2 * dim; ++f) {
      int ext[2];
      face_extent(c->hblocks[b], dim, f, ext);
      std::vector<unsigned char> cov((size_t)ext[0] * ext[1], 0);
      auto mark = [&](const int lo[2], const int hi[2]) -> bool {
        for (int t2 = lo[1]; t2 < hi[1]; ++t2)
          for (int t1 = lo[0]; t1 < hi[0]; ++t1)
            if (cov[(size_t)t2 * ext[0] + t1]++) return false;
        return true;
      };
      for (auto& p : c->hpatches)
        if (p.block == b && p.face == f && !mark(p.lo, p.hi))
          return fail(c, CFD_ERR_TOPOLOGY, "block %d face %d: overlapping boundary definitions", b, f);
      for (auto& h : c->hconns) {
        if (h.a == b && h.fa == f && !mark(h.loa, h.hia))
          return fail(c, CFD_ERR_TOPOLOGY, "block %d face %d: overlapping boundary definitions", b, f);
        if (h.b == b && h.fb == f && !mark(h.lob, h.hib))
          return fail(c, CFD_ERR_TOPOLOGY, "block %d face %d: overlapping boundary definitions", b, f);
      }
      for (auto v : cov)
        if (v == 0) return fail(c, CFD_ERR_TOPOLOGY, "block %d face %d has cells without a boundary condition", b, f);
    }
  }

  // --- block layout ---------------------------------------------------------
  c->blocks.resize(nb);
  long long cursor = 0, mcursor = 0, fcursor = 0, lcursor = 0, ccursor = 0, packed = 0, node0 = 0;
  const int nmet = dim * dim + 1;
  const int nfb = (2 * nv + 3) * dim;
  c->max_cells = c->max_padded = c->max_pos = 0;
  c->padded_total = 0;
  c->export_off.assign(nb, 0);
  for (int b = 0; b < nb; ++b) {
    const HBlock& h = c->hblocks[b];
    BlockDev& B = c->blocks[b];
    B.ni = h.ni;
    B.nj = h.nj;
    B.nk = h.nk;
    B.pi = (int)align_ll(h.ni + 4, 16);
    B.pj = h.nj + 4;
    const long long pk = dim == 3 ? h.nk + 4 : 1;
    const long long padded = (long long)B.pi * B.pj * pk;
    B.vstride = align_ll(padded, 16);
    // kernels address one array of a block with 32-bit byte offsets
    if (B.vstride * 8 >= (1LL << 32))
      return fail(c, CFD_ERR_UNSUPPORTED, "block %d: a padded array exceeds 4 GiB (%lld cells); split the block", b,
                  padded);
    const long long K = ((dim == 3 ? 2LL * B.pj : 0LL) + 2) * B.pi + 2;  // origin - array base
    // array base at cursor + 14 puts the origin (K = 2 mod 16) on a 16-double boundary
    B.origin = cursor + 14 + K;
    cursor = align_ll(cursor + 14 + (nv - 1) * B.vstride + padded, 16);
    B.morigin = mcursor + 14 + K;
    mcursor = align_ll(mcursor + 14 + (nmet - 1) * B.vstride + padded, 16);
    B.forigin = fcursor + 14 + K;
    fcursor = align_ll(fcursor + 14 + (nfb - 1) * B.vstride + padded, 16);
    B.corigin = 0;
    if (c->viscous) {
      // cell-centre coordinates
      B.corigin = ccursor + 14 + K;
      ccursor = align_ll(ccursor + 14 + (dim - 1) * B.vstride + padded, 16);
    }
    B.lorigin = 0;
    if (c->freezing) {
      B.lorigin = lcursor + 14 + K;
      lcursor = align_ll(lcursor + 14 + (dim * nv - 1) * B.vstride + padded, 16);
    }
    B.packed = packed;
    const long long ncell = (long long)h.ni * h.nj * h.nk;
    packed += ncell;
    B.node0 = node0;
    const long long nnode = (long long)(h.ni + 1) * (h.nj + 1) * (dim == 3 ? h.nk + 1 : 1);
    node0 += nnode;
    B.wall_mask = 0;
    B.wrap = 0;
    for (auto& p : c->hpatches)
      if (p.block == b && (p.kind == CFD_BC_SLIP_WALL || p.kind == CFD_BC_NOSLIP_WALL)) B.wall_mask |= 1 << p.face;
      else if (p.block == b && p.kind == CFD_BC_FARFIELD) {
        B.wall_mask |= FARFIELD_MASK_SHIFT << p.face;
        c->has_farfield = true;
      }
    c->max_cells = std::max(c->max_cells, ncell);
    const long long pe = (long long)(h.ni + 4) * (h.nj + 4) * (dim == 3 ? h.nk + 4 : 1);
    c->max_padded = std::max(c->max_padded, pe);
    c->export_off[b] = c->padded_total;
    c->padded_total += pe * nv;
    c->max_pos = std::max(c->max_pos, (long long)(h.ni + 1) * (h.nj + 1) * (dim == 3 ? h.nk + 1 : 1));
    c->max_nodes = c->max_pos;
    long long nfaces = (long long)(h.ni + 1) * h.nj * h.nk + (long long)h.ni * (h.nj + 1) * h.nk;
    if (dim == 3) nfaces += (long long)h.ni * h.nj * (h.nk + 1);
    c->max_faces = std::max(c->max_faces, nfaces);
  }
  for (auto& B : c->blocks) {
    B.ncell_total = packed;
    B.nnode_total = node0;
  }
  c->ncells = packed;
  c->nnodes = node0;
  c->state_doubles = cursor;
  c->metric_doubles = mcursor;
  c->facebar_doubles = fcursor;
  c->phi_doubles = lcursor;
  c->center_doubles = ccursor;

  // --- transfers, patches and ghost-fill chunks ------------------------------
  c->xfers.clear();
  long long xoff = 0;
  for (auto& h : c->hconns) {
    for (int dir = 0; dir < 2; ++dir) {
      TransferDev x{};
      const bool ab = dir == 0;  // receiver a, donor b
      x.rblock = ab ? h.a : h.b;
      x.rface = ab ? h.fa : h.fb;
      x.dblock = ab ? h.b : h.a;
      x.dface = ab ? h.fb : h.fa;
      const int* rlo = ab ? h.loa : h.lob;
      const int* rhi = ab ? h.hia : h.hib;
      const int* dlo = ab ? h.lob : h.loa;
      const int* dhi = ab ? h.hib : h.hia;
      x.rlo0 = rlo[0];
      x.rlo1 = rlo[1];
      x.len0 = rhi[0] - rlo[0];
      x.len1 = rhi[1] - rlo[1];
      x.dlo0 = dlo[0];
      x.dlo1 = dlo[1];
      x.dlen0 = dhi[0] - dlo[0];
      x.dlen1 = dhi[1] - dlo[1];
      x.orient = ab ? h.orient : inverse_orient(h.orient);
      x.buf = xoff;
      xoff += (long long)nv * NG * x.len0 * x.len1;
      c->xfers.push_back(x);
    }
  }
  c->xbuf_doubles = std::max(xoff, 16LL);
  c->patches.clear();
  for (auto& p : c->hpatches) {
    PatchDev d{};
    d.block = p.block;
    d.face = p.face;
    d.kind = p.kind;
    d.param = p.param_index;
    d.lo0 = p.lo[0];
    d.lo1 = p.lo[1];
    d.len0 = p.hi[0] - p.lo[0];
    d.len1 = p.hi[1] - p.lo[1];
    c->patches.push_back(d);
  }
  // phase 1 chunks sorted by owning block (pack: donor; patch: its block); phase 2 by receiver
  c->chunks1.clear();
  c->chunks2.clear();
  c->c1_begin.assign(nb + 1, 0);
  c->c2_begin.assign(nb + 1, 0);
  auto add_chunks = [](std::vector<ChunkDev>& v, int kind, int item, int count) {
    for (int s = 0; s < count; s += CHUNK) v.push_back(ChunkDev{kind, item, s, std::min(CHUNK, count - s)});
  };
  for (int b = 0; b < nb; ++b) {
    c->c1_begin[b] = (int)c->chunks1.size();
    for (size_t x = 0; x < c->xfers.size(); ++x)
      if (c->xfers[x].dblock == b) add_chunks(c->chunks1, 0, (int)x, NG * c->xfers[x].len0 * c->xfers[x].len1);
    for (size_t p = 0; p < c->patches.size(); ++p)
      if (c->patches[p].block == b) add_chunks(c->chunks1, 1, (int)p, NG * c->patches[p].len0 * c->patches[p].len1);
    c->c2_begin[b] = (int)c->chunks2.size();
    for (size_t x = 0; x < c->xfers.size(); ++x)
      if (c->xfers[x].rblock == b) add_chunks(c->chunks2, 2, (int)x, NG * c->xfers[x].len0 * c->xfers[x].len1);
  }
  c->c1_begin[nb] = (int)c->chunks1.size();
  c->c2_begin[nb] = (int)c->chunks2.size();
  // direct exchange: every connected ghost copied from the donor interior and
  // every physical patch, in one launch (per receiving block in per-block mode)
  c->chunksd.clear();
  c->cd_begin.assign(nb + 1, 0);
  for (int b = 0; b < nb; ++b) {
    c->cd_begin[b] = (int)c->chunksd.size();
    for (size_t x = 0; x < c->xfers.size(); ++x)
      if (c->xfers[x].rblock == b) add_chunks(c->chunksd, 3, (int)x, NG * c->xfers[x].len0 * c->xfers[x].len1);
    for (size_t p = 0; p < c->patches.size(); ++p)
      if (c->patches[p].block == b) add_chunks(c->chunksd, 1, (int)p, NG * c->patches[p].len0 * c->patches[p].len1);
  }
  c->cd_begin[nb] = (int)c->chunksd.size();
  // Axes along which a block is connected to itself end to end (opposite
  // faces, full ranges, no reorientation): the stage kernel reads the cells
  // that those ghosts copy, so the fill between the stages of a step leaves
  // these connections out (chunksw); every other reader fills in full.
  c->wrap_any = false;
  for (auto& h : c->hconns) {
    if (h.a != h.b || h.fa == h.fb || face_axis(h.fa) != face_axis(h.fb) || h.orient != 0) continue;
    const int ax = face_axis(h.fa);
    const HBlock& hb = c->hblocks[h.a];
    const int t1 = ax == 0 ? hb.nj : hb.ni, t2 = dim == 3 ? (ax == 2 ? hb.nj : hb.nk) : 1;
    const bool full = h.loa[0] == 0 && h.loa[1] == 0 && h.hia[0] == t1 && h.hia[1] == t2 && h.lob[0] == 0 &&
                      h.lob[1] == 0 && h.hib[0] == t1 && h.hib[1] == t2;
    if (!full) continue;
    c->blocks[h.a].wrap |= 1 << ax;
    c->wrap_any = true;
  }
  c->chunksw.clear();
  c->cw_begin.assign(nb + 1, 0);
  for (int b = 0; b < nb; ++b) {
    c->cw_begin[b] = (int)c->chunksw.size();
    for (size_t x = 0; x < c->xfers.size(); ++x) {
      const TransferDev& t = c->xfers[x];
      if (t.rblock != b) continue;
      const bool through = t.dblock == b && t.orient == 0 && (c->blocks[b].wrap >> (t.rface >> 1) & 1) &&
                           (t.rface >> 1) == (t.dface >> 1) && t.rface != t.dface;
      if (!through) add_chunks(c->chunksw, 3, (int)x, NG * t.len0 * t.len1);
    }
    for (size_t p = 0; p < c->patches.size(); ++p)
      if (c->patches[p].block == b) add_chunks(c->chunksw, 1, (int)p, NG * c->patches[p].len0 * c->patches[p].len1);
  }
  c->cw_begin[nb] = (int)c->chunksw.size();

  // --- tiles per variant -------------------------------------------------------
  int nvar_t = 0;
  const StageVariant* vars = stage_variants(dim, &nvar_t);
  c->nvariants = nvar_t;
  c->tiles_batched.assign(nvar_t, {});
  c->tiles_block.assign(nvar_t, {});
  c->tile_begin.assign(nvar_t, std::vector<int>(nb + 1, 0));
  for (int v = 0; v < nvar_t; ++v) {
    std::vector<TileDev> spatial;
    for (int b = 0; b < nb; ++b) {
      c->tile_begin[v][b] = (int)spatial.size();
      const BlockDev& B = c->blocks[b];
      const int kc = dim == 3 ? vars[v].kc : 1;
      const int nk = dim == 3 ? B.nk : 1;
      for (int k0 = 0; k0 < nk; k0 += kc)
        for (int j0 = 0; j0 < B.nj; j0 += vars[v].ty)
          for (int i0 = 0; i0 < B.ni; i0 += vars[v].tx) spatial.push_back(TileDev{b, i0, j0, k0});
    }
    c->tile_begin[v][nb] = (int)spatial.size();
    c->tiles_batched[v] = xcd_order(spatial, 0, spatial.size());
    std::vector<TileDev> per;
    for (int b = 0; b < nb; ++b) {
      auto part = xcd_order(spatial, c->tile_begin[v][b], c->tile_begin[v][b + 1]);
      per.insert(per.end(), part.begin(), part.end());
    }
    c->tiles_block[v] = per;
  }

  // --- workspace layout ---------------------------------------------------------
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1), ALIGN);
    return o;
  };
  c->off_stA = take(c->state_doubles * 8);
  c->off_stB = take(c->state_doubles * 8);
  c->off_stC = take(c->state_doubles * 8);
  if (c->cfg.rk_scheme == CFD_RK_CLASSIC4) {  // (inside the range zeroed at bind)
    c->off_rkD = take(c->state_doubles * 8);
    c->off_rkE = take(c->state_doubles * 8);
  }
  c->off_metric = take(c->metric_doubles * 8);
  c->off_nodes = take((size_t)c->nnodes * dim * 8);
  c->off_xbuf = take(c->xbuf_doubles * 8);
  c->off_inflow = take((size_t)std::max(c->nparam, 1) * MAXV * 8);
  c->off_dt = take(2 * 8);
  c->off_dtmin = take(8 * DT_SLOTS);
  c->off_err = take(4);
  c->off_normpart = take((size_t)cfd_ctx::NORM_PARTS * MAXV * 8);
  if (c->cfg.dt_mode == CFD_DT_LOCAL) c->off_dtloc = take((size_t)c->ncells * 8);
  if (c->freezing) c->off_phi = take((size_t)c->phi_doubles * 8);
  if (c->viscous) {
    c->vis_tiles.clear();
    {
      int vx, vy, vk;
      viscous_tile_shape(dim, &vx, &vy, &vk);
      for (int b = 0; b < nb; ++b)
        for (int k0 = 0; k0 < c->blocks[b].nk; k0 += vk)
          for (int j0 = 0; j0 < c->blocks[b].nj; j0 += vy)
            for (int i0 = 0; i0 < c->blocks[b].ni; i0 += vx) c->vis_tiles.push_back(TileDev{b, i0, j0, k0});
      // neighbouring tiles share halo cache lines: keep them on one XCD's L2
      c->vis_tiles = xcd_order(c->vis_tiles, 0, c->vis_tiles.size());
    }
    c->off_vistiles = take(std::max<size_t>(c->vis_tiles.size(), 1) * sizeof(TileDev));
    c->off_centers = take((size_t)c->center_doubles * 8);
    c->off_npos = take((size_t)c->nnodes * dim * 8);
    c->off_rv = take((size_t)c->ncells * (dim + 1) * 8);
  }
  c->off_blocks = take(c->blocks.size() * sizeof(BlockDev));
  c->off_xfers = take(c->xfers.size() * sizeof(TransferDev));
  c->off_patches = take(c->patches.size() * sizeof(PatchDev));
  c->off_chunks1 = take(c->chunks1.size() * sizeof(ChunkDev));
  c->off_chunks2 = take(c->chunks2.size() * sizeof(ChunkDev));
  c->off_chunksd = take(c->chunksd.size() * sizeof(ChunkDev));
  c->off_chunksw = take(c->chunksw.size() * sizeof(ChunkDev));
  c->off_export = take(c->export_off.size() * sizeof(long long));
  c->off_tiles_batched.assign(nvar_t, 0);
  c->off_tiles_block.assign(nvar_t, 0);
  for (int v = 0; v < nvar_t; ++v) {
    c->off_tiles_batched[v] = take(c->tiles_batched[v].size() * sizeof(TileDev));
    c->off_tiles_block[v] = take(c->tiles_block[v].size() * sizeof(TileDev));
  }
  if (c->adjoint) {
    // per block face and tangential position, the item whose ghost cells
    // copy that position's cells: a transfer (this block as donor) or a patch
    const int nf = 2 * dim;
    c->fmap_off.assign((size_t)nb * 6, 0);
    c->facemap.clear();
    auto t1ext = [&](int b, int f) { return (f >> 1) == 0 ? c->blocks[b].nj : c->blocks[b].ni; };
    auto t2ext = [&](int b, int f) { return dim == 3 ? ((f >> 1) == 2 ? c->blocks[b].nj : c->blocks[b].nk) : 1; };
    for (int b = 0; b < nb; ++b)
      for (int f = 0; f < nf; ++f) {
        c->fmap_off[(size_t)b * 6 + f] = (long long)c->facemap.size();
        c->max_face_area = std::max(c->max_face_area, (long long)t1ext(b, f) * t2ext(b, f));
        c->facemap.resize(c->facemap.size() + (size_t)t1ext(b, f) * t2ext(b, f), FMAP_NONE);
      }
    for (size_t x = 0; x < c->xfers.size(); ++x) {
      const TransferDev& X = c->xfers[x];
      const long long base = c->fmap_off[(size_t)X.dblock * 6 + X.dface];
      const int T1 = t1ext(X.dblock, X.dface);
      for (int r2 = 0; r2 < X.len1; ++r2)
        for (int r1 = 0; r1 < X.len0; ++r1) {
          int d1, d2;
          orient_map(X.orient, r1, r2, X.dlen0, X.dlen1, d1, d2);
          c->facemap[base + (X.dlo0 + d1) + (long long)(X.dlo1 + d2) * T1] = (int)x;
        }
    }
    for (size_t p = 0; p < c->patches.size(); ++p) {
      const PatchDev& P = c->patches[p];
      const long long base = c->fmap_off[(size_t)P.block * 6 + P.face];
      const int T1 = t1ext(P.block, P.face);
      for (int e1 = 0; e1 < P.len1; ++e1)
        for (int e0 = 0; e0 < P.len0; ++e0)
          c->facemap[base + (P.lo0 + e0) + (long long)(P.lo1 + e1) * T1] = -(int)p - 1;
    }
    // 2D: the tile pass finalizes cells next to physical patches itself; the
    // boundary gather is needed for connections and for blocks whose last
    // two cells along an axis fall into different tiles
    c->need_bgather = dim == 3 || !c->xfers.empty();
    if (dim == 2)
      for (int b = 0; b < nb; ++b)
        if (c->blocks[b].ni % VJP_TILE == 1 || c->blocks[b].nj % VJP_TILE == 1) c->need_bgather = true;
    c->vtiles.clear();
    if (dim == 2)
      for (int b = 0; b < nb; ++b)
        for (int j0 = 0; j0 < c->blocks[b].nj; j0 += VJP_TILE)
          for (int i0 = 0; i0 < c->blocks[b].ni; i0 += VJP_TILE) c->vtiles.push_back(TileDev{b, i0, j0, 0});
    // XCD-aware order (each tile writes only its own outputs, so the order
    // changes no result)
    if (!c->vtiles.empty()) c->vtiles = xcd_order(c->vtiles, 0, c->vtiles.size());
    c->obj_chunks.clear();
    c->obj_begin.assign(nf + 1, 0);
    for (int f = 0; f < nf; ++f) {
      c->obj_begin[f] = (int)c->obj_chunks.size();
      for (size_t p = 0; p < c->patches.size(); ++p)
        if (c->patches[p].face == f && c->patches[p].kind == PK_SLIP_WALL)
          add_chunks(c->obj_chunks, 1, (int)p, c->patches[p].len0 * c->patches[p].len1);
    }
    c->obj_begin[nf] = (int)c->obj_chunks.size();
    c->part_off.assign(c->patches.size(), 0);
    c->inflow_list.clear();
    c->wall_list.clear();
    long long po = 0;
    for (size_t p = 0; p < c->patches.size(); ++p) {
      c->part_off[p] = po;
      po += (long long)nv * c->patches[p].len0 * c->patches[p].len1;
      if (c->patches[p].kind == PK_SUP_INFLOW) c->inflow_list.push_back((int)p);
      if (c->patches[p].kind == PK_SLIP_WALL) c->wall_list.push_back((int)p);
    }
    c->part_doubles = std::max(po, 16LL);
    c->off_stD = take(c->state_doubles * 8);
    c->off_qbar = take(c->state_doubles * 8);
    c->off_facebar = take(c->facebar_doubles * 8);
    c->off_metricbar = take(c->metric_doubles * 8);
    c->off_G = take((size_t)nv * c->ncells * 8);
    c->off_T = take((size_t)nv * c->ncells * 8);
    c->off_thetabar = take((size_t)std::max(c->nparam, 1) * MAXV * 8);
    c->off_part = take(c->part_doubles * 8);
    c->off_partoff = take(c->part_off.size() * sizeof(long long));
    c->off_facemap = take(c->facemap.size() * sizeof(int));
    c->off_fmapoff = take(c->fmap_off.size() * sizeof(long long));
    c->off_vtiles = take(std::max<size_t>(c->vtiles.size(), 1) * sizeof(TileDev));
    c->off_objchunks = take(c->obj_chunks.size() * sizeof(ChunkDev));
    c->off_inflowlist = take(c->inflow_list.size() * sizeof(int));
    c->off_walllist = take(c->wall_list.size() * sizeof(int));
    c->off_sumpart = take((size_t)cfd_ctx::SUM_PARTS * MAXV * 8);
    c->off_J = take(8);
  }
  c->ws_bytes = off;
  c->finalized = true;
  if (ws_bytes) *ws_bytes = off;
  return CFD_OK;
}

// ---------------------------------------------------------------------------

static ViscArgs visc_args(cfd_ctx* c, const double* q) {
  ViscArgs v{};
  v.blocks = c->dptr<BlockDev>(c->off_blocks);
  v.xfers = c->dptr<TransferDev>(c->off_xfers);
  v.patches = c->dptr<PatchDev>(c->off_patches);
  v.chunks = c->dptr<ChunkDev>(c->off_chunks1);
  v.nodes = c->dptr<double>(c->off_nodes);
  v.metric = c->metric();
  v.centers = c->dptr<double>(c->off_centers);
  v.npos = c->dptr<double>(c->off_npos);
  v.q = q;
  v.rv = c->dptr<double>(c->off_rv);
  v.mu = c->cfg.viscosity;
  v.kcond = c->cfg.viscosity > 0.0 ? c->cfg.viscosity / ((c->cfg.gamma - 1.0) * c->cfg.prandtl) : 0.0;
  v.gamma = c->cfg.gamma;
  v.tiles = c->dptr<TileDev>(c->off_vistiles);
  v.ntiles = (int)c->vis_tiles.size();
  v.wrap = 1;
  return v;
}

static double visc_cv(const cfd_ctx* c) {
  if (!c->viscous) return 0.0;
  return 4.0 * std::max(4.0 / 3.0, c->cfg.gamma / c->cfg.prandtl) * c->cfg.viscosity;
}

static cfd_status recompute_metrics(cfd_ctx* c) {
  HIP_TRY(c, hipMemsetAsync(c->dptr<int>(c->off_err), 0, sizeof(int), c->stream));
  MetricArgs m{c->dptr<BlockDev>(c->off_blocks), c->dptr<double>(c->off_nodes), c->metric(), c->dptr<int>(c->off_err)};
  HIP_TRY(c, launch_metrics(c->dim, m, c->max_pos, (int)c->blocks.size(), c->stream));
  int err = 0;
  HIP_TRY(c, hipMemcpyAsync(&err, c->dptr<int>(c->off_err), sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (err) return fail(c, CFD_ERR_GRID, "grid has a non-positive or non-finite cell volume");
  c->dt_valid = false;
  if (c->viscous) {
    // cell centres, their first ghost layer (all interior centres first), pseudo-node positions
    ViscArgs v = visc_args(c, nullptr);
    const int nb = (int)c->blocks.size();
    HIP_TRY(c, launch_cell_centers(c->dim, v, c->max_cells, nb, c->stream));
    HIP_TRY(c, launch_ghost_centers(c->dim, v, (int)c->chunks1.size(), c->stream));
    HIP_TRY(c, launch_pseudo_nodes(c->dim, v, c->max_nodes, nb, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  return CFD_OK;
}

template <class T>
static cfd_status upload(cfd_ctx* c, size_t off, const std::vector<T>& v) {
  if (v.empty()) return CFD_OK;
  HIP_TRY(c, hipMemcpyAsync(c->ws + off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  return CFD_OK;
}

extern "C" cfd_status cfd_bind_workspace(cfd_ctx* c, void* ptr, size_t bytes) {
  cfd_status s = need(c, true, false);
  if (s != CFD_OK) return s;
  if (c->device < 0) return fail(c, CFD_ERR_HIP, "no HIP device was available when the context was created");
  if (!ptr || bytes < c->ws_bytes) return fail(c, CFD_ERR_ARG, "workspace too small (%zu < %zu)", bytes, c->ws_bytes);
  if (reinterpret_cast<uintptr_t>(ptr) % ALIGN) return fail(c, CFD_ERR_ARG, "workspace must be %zu-byte aligned", ALIGN);
  release_graph(c);
  c->ws = static_cast<char*>(ptr);
  c->bound = true;
  // the state buffers start zeroed so unused padding never holds NaN patterns
  HIP_TRY(c, hipMemsetAsync(c->ws + c->off_stA, 0, c->off_nodes - c->off_stA, c->stream));
  // tables
  if ((s = upload(c, c->off_blocks, c->blocks)) != CFD_OK) return s;
  if ((s = upload(c, c->off_xfers, c->xfers)) != CFD_OK) return s;
  if ((s = upload(c, c->off_patches, c->patches)) != CFD_OK) return s;
  if ((s = upload(c, c->off_chunks1, c->chunks1)) != CFD_OK) return s;
  if ((s = upload(c, c->off_chunks2, c->chunks2)) != CFD_OK) return s;
  if ((s = upload(c, c->off_chunksd, c->chunksd)) != CFD_OK) return s;
  if ((s = upload(c, c->off_chunksw, c->chunksw)) != CFD_OK) return s;
  if ((s = upload(c, c->off_export, c->export_off)) != CFD_OK) return s;
  for (int v = 0; v < c->nvariants; ++v) {
    if ((s = upload(c, c->off_tiles_batched[v], c->tiles_batched[v])) != CFD_OK) return s;
    if ((s = upload(c, c->off_tiles_block[v], c->tiles_block[v])) != CFD_OK) return s;
  }
  if (c->adjoint) {
    if ((s = upload(c, c->off_partoff, c->part_off)) != CFD_OK) return s;
    if ((s = upload(c, c->off_facemap, c->facemap)) != CFD_OK) return s;
    if ((s = upload(c, c->off_fmapoff, c->fmap_off)) != CFD_OK) return s;
    if ((s = upload(c, c->off_vtiles, c->vtiles)) != CFD_OK) return s;
    if ((s = upload(c, c->off_objchunks, c->obj_chunks)) != CFD_OK) return s;
    if ((s = upload(c, c->off_inflowlist, c->inflow_list)) != CFD_OK) return s;
    if ((s = upload(c, c->off_walllist, c->wall_list)) != CFD_OK) return s;
    HIP_TRY(c, hipMemsetAsync(c->ws + c->off_stD, 0, c->off_G - c->off_stD, c->stream));
  }
  if (c->viscous && (s = upload(c, c->off_vistiles, c->vis_tiles)) != CFD_OK) return s;
  // nodes: [coord][concatenated nodes]
  std::vector<double> nodes((size_t)c->nnodes * c->dim);
  for (size_t b = 0; b < c->hblocks.size(); ++b) {
    const HBlock& h = c->hblocks[b];
    const size_t nn = h.nodes.size() / c->dim;
    for (int cc = 0; cc < c->dim; ++cc)
      std::memcpy(&nodes[cc * c->nnodes + c->blocks[b].node0], &h.nodes[cc * nn], nn * 8);
  }
  if ((s = upload(c, c->off_nodes, nodes)) != CFD_OK) return s;
  std::vector<double> bcp((size_t)std::max(c->nparam, 1) * MAXV, 0.0);
  for (auto& p : c->hpatches)
    if (p.param_index >= 0)
      for (int v = 0; v < MAXV; ++v) bcp[(size_t)p.param_index * MAXV + v] = p.params[v];
  if ((s = upload(c, c->off_inflow, bcp)) != CFD_OK) return s;
  std::vector<double> dt = {c->cfg.dt_mode == CFD_DT_FIXED ? c->cfg.dt_fixed : 0.0, 0.0};
  if ((s = upload(c, c->off_dt, dt)) != CFD_OK) return s;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return recompute_metrics(c);
}

extern "C" cfd_status cfd_set_nodes(cfd_ctx* c, const double* dev_nodes) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (!dev_nodes) return CFD_ERR_ARG;
  HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_nodes, dev_nodes, (size_t)c->nnodes * c->dim * 8,
                            hipMemcpyDeviceToDevice, c->stream));
  return recompute_metrics(c);
}

extern "C" cfd_status cfd_set_bc_params(cfd_ctx* c, int patch_id, const double* params) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (patch_id < 0 || patch_id >= (int)c->hpatches.size() || !params) return CFD_ERR_ARG;
  HPatch& p = c->hpatches[patch_id];
  if (!has_params(p.kind)) return fail(c, CFD_ERR_ARG, "patch %d has no parameters", patch_id);
  double tmp[MAXV];
  if ((s = check_params(c, p.kind, params, tmp)) != CFD_OK) return s;
  for (int v = 0; v < MAXV; ++v) p.params[v] = tmp[v];
  HIP_TRY(c, hipMemcpyAsync(c->dptr<double>(c->off_inflow) + (size_t)p.param_index * MAXV, tmp, sizeof tmp,
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return CFD_OK;
}

// ---------------------------------------------------------------------------
// launch helpers

static CellArgs cell_args(cfd_ctx* c) {
  CellArgs a{};
  a.blocks = c->dptr<BlockDev>(c->off_blocks);
  a.metric = c->metric();
  a.offsets = c->dptr<long long>(c->off_export);
  a.dtmin = c->dptr<unsigned long long>(c->off_dtmin);
  a.err = c->dptr<int>(c->off_err);
  a.gas = make_gas(c->cfg.gamma);
  a.visc_cv = visc_cv(c);
  return a;
}

static GhostArgs ghost_args(cfd_ctx* c, double* q) {
  GhostArgs g{};
  g.blocks = c->dptr<BlockDev>(c->off_blocks);
  g.xfers = c->dptr<TransferDev>(c->off_xfers);
  g.patches = c->dptr<PatchDev>(c->off_patches);
  g.q = q;
  g.buf = c->dptr<double>(c->off_xbuf);
  g.bcparams = c->dptr<double>(c->off_inflow);
  g.metric = c->metric();
  g.gas = make_gas(c->cfg.gamma);
  return g;
}

static StageArgs stage_args(cfd_ctx* c) {
  StageArgs a{};
  a.blocks = c->dptr<BlockDev>(c->off_blocks);
  a.patches = c->dptr<PatchDev>(c->off_patches);
  a.npatches = (int)c->patches.size();
  a.metric = c->metric();
  a.dt = c->dptr<double>(c->off_dt);
  a.gas = make_gas(c->cfg.gamma);
  a.half_eps = 0.5 * c->cfg.muscl_eps;
  a.kappa = c->cfg.muscl_kappa;
  a.efix = c->cfg.efix;
  a.half_inv_efix = c->cfg.efix > 0.0 ? 0.5 / c->cfg.efix : 0.0;
  for (int v = 0; v < MAXV; ++v) a.e2[v] = c->cfg.lim_eps[v] * c->cfg.lim_eps[v];
  a.dtloc = c->cfg.dt_mode == CFD_DT_LOCAL ? c->dptr<double>(c->off_dtloc) : nullptr;
  a.cfl = c->cfg.cfl;
  a.phi = c->frozen ? c->dptr<double>(c->off_phi) : nullptr;
  a.rv = c->viscous ? c->dptr<double>(c->off_rv) : nullptr;
  a.visc_cv = visc_cv(c);
  a.wrap = c->frozen ? 0 : 1;  // (the frozen factors of ghost cells are read at the ghosts)
  return a;
}

static cfd_status fill_ghosts(cfd_ctx* c, double* q, hipStream_t s, bool stencil_only = false,
                              bool* promote = nullptr);

// Ghost fill of state buffer q and, for the Navier-Stokes equations, the
// viscous residual of q that the next stage-kernel launch subtracts.
// stencil_only: q is read by the stage kernel and the viscous pass alone (see
// fill_ghosts); promote: see fill_ghosts.
static cfd_status stage_prep(cfd_ctx* c, double* q, hipStream_t s, bool stencil_only = false,
                             bool* promote = nullptr) {
  cfd_status st = fill_ghosts(c, q, s, stencil_only, promote);
  if (st != CFD_OK || !c->viscous) return st;
  ViscArgs v = visc_args(c, q);
  HIP_TRY(c, launch_viscous(c->dim, v, s));
  return CFD_OK;
}

// Fill every ghost layer of state buffer q: pack + physical patches, then
// unpack (packed mode), or direct copies + physical patches (direct mode).
// stencil_only (direct mode): q is read by the stage kernel and the viscous
// pass alone, which read the periodic neighbours of a self-connected axis
// through the wrap, so those connections are left out (their ghosts keep older
// values, or NaN with CFD_NAN_GHOSTS).
// promote (non-null and true): the first ghost launch also forms the step's
// time step from the slots (the work of dt_promote_kernel) and *promote is
// cleared; it stays set when nothing is launched.
static cfd_status fill_ghosts(cfd_ctx* c, double* q, hipStream_t s, bool stencil_only, bool* promote) {
  GhostArgs g = ghost_args(c, q);
  const int nb = (int)c->blocks.size();
  auto launch = [&](int n) -> hipError_t {
    if (n <= 0 || !promote || !*promote) return launch_ghost(c->dim, g, n, s);
    GhostArgs gp = g;
    gp.dt = c->dptr<double>(c->off_dt);
    gp.dtmin = c->dptr<unsigned long long>(c->off_dtmin);
    gp.cfl = c->cfg.cfl;
    *promote = false;
    return launch_ghost(c->dim, gp, n, s);
  };
  if (c->cfg.debug_flags & CFD_NAN_GHOSTS) {
    CellArgs n = cell_args(c);
    n.dst = q;
    HIP_TRY(c, launch_nan_ghosts(c->dim, n, c->max_padded, nb, s));
  }
  if (c->ghost_mode == CFD_GHOSTS_DIRECT) {
    const bool w = stencil_only && c->wrap_any;
    g.chunks = c->dptr<ChunkDev>(w ? c->off_chunksw : c->off_chunksd);
    const std::vector<int>& begin = w ? c->cw_begin : c->cd_begin;
    if (c->exec_mode == CFD_EXEC_PER_BLOCK) {
      for (int b = 0; b < nb; ++b) {
        g.chunk_begin = begin[b];
        HIP_TRY(c, launch(begin[b + 1] - begin[b]));
      }
    } else {
      g.chunk_begin = 0;
      HIP_TRY(c, launch(begin[nb]));
    }
    return CFD_OK;
  }
  if (c->exec_mode == CFD_EXEC_PER_BLOCK) {
    g.chunks = c->dptr<ChunkDev>(c->off_chunks1);
    for (int b = 0; b < nb; ++b) {
      g.chunk_begin = c->c1_begin[b];
      HIP_TRY(c, launch(c->c1_begin[b + 1] - c->c1_begin[b]));
    }
    g.chunks = c->dptr<ChunkDev>(c->off_chunks2);
    for (int b = 0; b < nb; ++b) {
      g.chunk_begin = c->c2_begin[b];
      HIP_TRY(c, launch(c->c2_begin[b + 1] - c->c2_begin[b]));
    }
  } else {
    g.chunks = c->dptr<ChunkDev>(c->off_chunks1);
    g.chunk_begin = 0;
    HIP_TRY(c, launch((int)c->chunks1.size()));
    g.chunks = c->dptr<ChunkDev>(c->off_chunks2);
    HIP_TRY(c, launch((int)c->chunks2.size()));
  }
  return CFD_OK;
}

static EventPair& next_event(cfd_ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    EventPair e{};
    (void)hipEventCreate(&e.a);
    (void)hipEventCreate(&e.b);
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

// Limiter instantiation of the stage kernel: frozen factors, van Albada with
// every regularisation zero (the specialisation without e^2), or the
// configured limiter.
static int stage_limiter(const cfd_ctx* c) {
  if (c->frozen) return LIM_FROZEN;
  if (c->cfg.limiter == CFD_LIM_VANALBADA) {
    bool zero = true;
    for (int v = 0; v < c->nvar; ++v) zero = zero && c->cfg.lim_eps[v] == 0.0;
    if (zero) return LIM_VANALBADA0;
  }
  return c->cfg.limiter;
}

static cfd_status launch_stage_all(cfd_ctx* c, StageArgs a, hipStream_t s, bool timed) {
  const int v = c->variant;
  const int nb = (int)c->blocks.size();
  EventPair* ev = nullptr;
  if (timed) {
    ev = &next_event(c);
    HIP_TRY(c, hipEventRecord(ev->a, s));
  }
  if (c->exec_mode == CFD_EXEC_PER_BLOCK) {
    a.tiles = c->dptr<TileDev>(c->off_tiles_block[v]);
    for (int b = 0; b < nb; ++b) {
      a.tile_begin = c->tile_begin[v][b];
      a.tile_end = c->tile_begin[v][b + 1];
      HIP_TRY(c, launch_stage(c->dim, c->cfg.flux, stage_limiter(c), v, c->has_farfield, a,
                              a.tile_end - a.tile_begin, false, s));
    }
  } else {
    a.tiles = c->dptr<TileDev>(c->off_tiles_batched[v]);
    a.tile_begin = 0;
    a.tile_end = (int)c->tiles_batched[v].size();
    HIP_TRY(c, launch_stage(c->dim, c->cfg.flux, stage_limiter(c), v, c->has_farfield, a,
                            a.tile_end, c->exec_mode == CFD_EXEC_PERSISTENT, s));
  }
  if (timed) {
    HIP_TRY(c, hipEventRecord(ev->b, s));
    c->prof_launches += 1;
  }
  return CFD_OK;
}

// dt <- cfl * (minimum over the time-step slots), slots <- +inf, in a launch of its own
static hipError_t launch_promote(cfd_ctx* c, hipStream_t s) {
  return launch_dt_promote(c->dptr<double>(c->off_dt), c->dptr<unsigned long long>(c->off_dtmin), c->cfg.cfl, 1,
                           nullptr, s);
}

// Classical fourth-order Runge-Kutta step (CFD_RK_CLASSIC4): the stage kernel
// writes Y2 = Q - dt/2 R(Q) into B, Y3 = Q - dt/2 R(Y2) into C,
// Y4 = Q - dt R(Y3) into D and Z = Q - dt/6 R(Y4) into E; the combination
// kernel forms Q^(n+1) in A, and the next step's Omega/lambda comes from it
// (the cell time-step kernel, in place of the stage kernel's epilogue).
static cfd_status enqueue_classic4(cfd_ctx* c, hipStream_t s, bool timed, bool promote) {
  double* A = c->stA();
  double* buf[5] = {A, c->stB(), c->stC(), c->dptr<double>(c->off_rkD), c->dptr<double>(c->off_rkE)};
  const double alpha[4] = {0.5, 0.5, 1.0, 1.0 / 6.0};
  for (int k = 0; k < 4; ++k) {
    cfd_status st = stage_prep(c, buf[k], s, !c->frozen, k == 0 ? &promote : nullptr);
    if (st != CFD_OK) return st;
    if (k == 0 && promote) HIP_TRY(c, launch_promote(c, s));
    StageArgs a = stage_args(c);
    a.qin = buf[k];
    a.q0 = A;
    a.qout = buf[k + 1];
    a.mode = MODE_STAGE;
    a.alpha = alpha[k];
    a.dtmin = nullptr;
    if ((st = launch_stage_all(c, a, s, timed)) != CFD_OK) return st;
  }
  Rk4Args r{};
  r.blocks = c->dptr<BlockDev>(c->off_blocks);
  r.q = A;
  r.y2 = buf[1];
  r.y3 = buf[2];
  r.y4 = buf[3];
  r.z = buf[4];
  r.out = A;
  r.gas = make_gas(c->cfg.gamma);
  const int nb = (int)c->blocks.size();
  HIP_TRY(c, launch_rk4_combine(c->dim, r, c->max_cells, nb, s));
  CellArgs ca = cell_args(c);
  if (c->cfg.debug_flags & CFD_CHECK_FINITE) {
    for (int k = 1; k < 5; ++k) {
      ca.src = buf[k];
      HIP_TRY(c, launch_check_state(c->dim, ca, c->max_cells, nb, s));
    }
    ca.src = A;
    HIP_TRY(c, launch_check_state(c->dim, ca, c->max_cells, nb, s));
  }
  if (c->cfg.dt_mode != CFD_DT_FIXED) {  // (the step's dt_promote left dtmin at +inf)
    ca.src = A;
    if (c->cfg.dt_mode == CFD_DT_LOCAL) {
      ca.dtloc = c->dptr<double>(c->off_dtloc);
      ca.cfl = c->cfg.cfl;
    }
    HIP_TRY(c, launch_cell_dt(c->dim, ca, c->max_cells, nb, s));
  }
  return CFD_OK;
}

// Enqueue one full Runge-Kutta step on stream s.
static cfd_status enqueue_step(cfd_ctx* c, hipStream_t s, bool timed) {
  const bool cfl = c->cfg.dt_mode != CFD_DT_FIXED;
  // (with the CFL step, the previous step's minimum becomes this step's dt in
  // the first ghost launch, or in its own launch when the first stage input
  // needs no ghost fill; either way before the first stage kernel)
  bool promote = cfl;
  if (c->cfg.rk_scheme == CFD_RK_CLASSIC4) return enqueue_classic4(c, s, timed, promote);
  const int M = c->cfg.rk_stages;
  double* A = c->stA();
  double* Bf = c->stB();
  double* Cf = c->stC();
  double* in = A;
  for (int k = 1; k <= M; ++k) {
    // (a single stage writes into B and is copied back: the kernel reads its
    // input's neighbours while writing, so it never updates in place)
    double* out = (k == M && M > 1) ? A : ((k % 2) ? Bf : Cf);
    // (an unfrozen step reads its stage inputs in the stage kernel and the
    // viscous pass only, both of which read periodic neighbours through the wrap)
    cfd_status st = stage_prep(c, in, s, !c->frozen, k == 1 ? &promote : nullptr);
    if (st != CFD_OK) return st;
    if (k == 1 && promote) HIP_TRY(c, launch_promote(c, s));
    StageArgs a = stage_args(c);
    a.qin = in;
    a.q0 = A;
    a.qout = out;
    a.mode = MODE_STAGE;
    a.alpha = 1.0 / (double)(M - k + 1);
    a.dtmin = (k == M && cfl) ? c->dptr<unsigned long long>(c->off_dtmin) : nullptr;
    st = launch_stage_all(c, a, s, timed);
    if (st != CFD_OK) return st;
    if (c->cfg.debug_flags & CFD_CHECK_FINITE) {
      CellArgs ca = cell_args(c);
      ca.src = out;
      HIP_TRY(c, launch_check_state(c->dim, ca, c->max_cells, (int)c->blocks.size(), s));
    }
    in = out;
  }
  if (M == 1) HIP_TRY(c, hipMemcpyAsync(A, Bf, (size_t)c->state_doubles * 8, hipMemcpyDeviceToDevice, s));
  return CFD_OK;
}

// CFD_CHECK_FINITE: clear the device error flag / read it back (synchronises).
static cfd_status debug_clear(cfd_ctx* c) {
  HIP_TRY(c, hipMemsetAsync(c->dptr<int>(c->off_err), 0, sizeof(int), c->stream));
  return CFD_OK;
}
static cfd_status debug_flagged(cfd_ctx* c, bool* bad) {
  int err = 0;
  HIP_TRY(c, hipMemcpyAsync(&err, c->dptr<int>(c->off_err), sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *bad = err != 0;
  return CFD_OK;
}

static cfd_status ensure_dt(cfd_ctx* c) {
  if (c->cfg.dt_mode == CFD_DT_FIXED || c->dt_valid) return CFD_OK;
  HIP_TRY(c, launch_set_u64(c->dptr<unsigned long long>(c->off_dtmin), 0x7ff0000000000000ULL, DT_SLOTS, c->stream));
  CellArgs a = cell_args(c);
  a.src = c->stA();
  if (c->cfg.dt_mode == CFD_DT_LOCAL) {
    a.dtloc = c->dptr<double>(c->off_dtloc);
    a.cfl = c->cfg.cfl;
  }
  HIP_TRY(c, launch_cell_dt(c->dim, a, c->max_cells, (int)c->blocks.size(), c->stream));
  c->dt_valid = true;
  return CFD_OK;
}

static cfd_status build_graph(cfd_ctx* c) {
  release_graph(c);
  if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  cfd_status st = enqueue_step(c, c->cap_stream, false);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
  if (st != CFD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(c, CFD_ERR_HIP, "stream capture: %s", hipGetErrorString(e));
  c->graph = g;
  HIP_TRY(c, hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
  c->graph_valid = true;
  return CFD_OK;
}

// ---------------------------------------------------------------------------

static cfd_status set_state_impl(cfd_ctx* c, const double* src, int primitive) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (!src) return CFD_ERR_ARG;
  HIP_TRY(c, hipMemsetAsync(c->dptr<int>(c->off_err), 0, sizeof(int), c->stream));
  CellArgs a = cell_args(c);
  a.src = src;
  a.dst = c->stA();
  a.flag_primitive = primitive;
  HIP_TRY(c, launch_set_state(c->dim, a, c->max_cells, (int)c->blocks.size(), c->stream));
  int err = 0;
  HIP_TRY(c, hipMemcpyAsync(&err, c->dptr<int>(c->off_err), sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (err) return fail(c, CFD_ERR_NONFINITE, "state has a non-positive or non-finite density or pressure");
  c->have_state = true;
  c->dt_valid = false;
  return ensure_dt(c);
}

extern "C" cfd_status cfd_set_state(cfd_ctx* c, const double* dev_Q) { return set_state_impl(c, dev_Q, 0); }
extern "C" cfd_status cfd_set_state_primitive(cfd_ctx* c, const double* dev_q) { return set_state_impl(c, dev_q, 1); }

extern "C" cfd_status cfd_get_state(cfd_ctx* c, double* dev_Q) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (!dev_Q) return CFD_ERR_ARG;
  CellArgs a = cell_args(c);
  a.src = c->stA();
  a.dst = dev_Q;
  HIP_TRY(c, launch_get_state(c->dim, a, c->max_cells, (int)c->blocks.size(), c->stream));
  return CFD_OK;
}

extern "C" cfd_status cfd_residual(cfd_ctx* c, double* dev_R) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (!dev_R) return CFD_ERR_ARG;
  if (!c->have_state) return fail(c, CFD_ERR_STATE, "no state set");
  s = stage_prep(c, c->stA(), c->stream);
  if (s != CFD_OK) return s;
  StageArgs a = stage_args(c);
  a.qin = c->stA();
  a.q0 = c->stA();
  a.qout = nullptr;
  a.Rout = dev_R;
  a.mode = MODE_RESIDUAL;
  if ((s = launch_stage_all(c, a, c->stream, false)) != CFD_OK) return s;
  if (c->cfg.debug_flags & CFD_CHECK_FINITE) {
    bool bad = false;
    if ((s = debug_clear(c)) != CFD_OK) return s;
    HIP_TRY(c, launch_check_packed(dev_R, (long long)c->nvar * c->ncells, c->dptr<int>(c->off_err), c->stream));
    if ((s = debug_flagged(c, &bad)) != CFD_OK) return s;
    if (bad) return fail(c, CFD_ERR_NONFINITE, "the residual has a non-finite entry");
  }
  return CFD_OK;
}

extern "C" cfd_status cfd_residual_norms(cfd_ctx* c, double* dev_R, double* dev_norms) {
  if (!dev_norms) return CFD_ERR_ARG;
  cfd_status s = cfd_residual(c, dev_R);
  if (s != CFD_OK) return s;
  const int parts = (int)std::min<long long>(cfd_ctx::NORM_PARTS, std::max<long long>(1, c->ncells / 4096));
  HIP_TRY(c, launch_sumsq(c->nvar, dev_R, c->ncells, c->dptr<double>(c->off_normpart), parts, dev_norms, c->stream));
  return CFD_OK;
}

extern "C" cfd_status cfd_residual_norms_noalloc(cfd_ctx* c, double* dev_R, double* dev_norms) {
  if (!dev_norms || !dev_R) return CFD_ERR_ARG;
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  double* part = scratch_of(c->device);
  if (!part) return fail(c, CFD_ERR_HIP, "the library scratch has no device address on device %d", c->device);
  const int parts = (int)std::min<long long>(cfd_ctx::NORM_PARTS, std::max<long long>(1, c->ncells / 4096));
  if ((long long)parts * c->nvar > SCRATCH_DOUBLES)
    return fail(c, CFD_ERR_UNSUPPORTED, "%d partial sums exceed the library scratch of %d doubles", parts * c->nvar,
                SCRATCH_DOUBLES);
  if ((s = cfd_residual(c, dev_R)) != CFD_OK) return s;
  // every partial slot [v][part] is written before it is read: nothing to clear
  HIP_TRY(c, launch_sumsq(c->nvar, dev_R, c->ncells, part, parts, dev_norms, c->stream));
  return CFD_OK;
}

extern "C" cfd_status cfd_time_step(cfd_ctx* c, double* dev_dt) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (!dev_dt) return CFD_ERR_ARG;
  if (!c->have_state) return fail(c, CFD_ERR_STATE, "no state set");
  if (c->cfg.dt_mode == CFD_DT_FIXED) {
    HIP_TRY(c, launch_copy_dt(c->dptr<double>(c->off_dt), dev_dt, c->stream));
    return CFD_OK;
  }
  if ((s = ensure_dt(c)) != CFD_OK) return s;
  HIP_TRY(c, launch_dt_promote(c->dptr<double>(c->off_dt), c->dptr<unsigned long long>(c->off_dtmin), c->cfg.cfl, 0,
                               dev_dt, c->stream));
  return CFD_OK;
}

extern "C" cfd_status cfd_rk_step(cfd_ctx* c, int nsteps, double* dev_dt_last) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (nsteps < 0) return CFD_ERR_ARG;
  if (!c->have_state) return fail(c, CFD_ERR_STATE, "no state set");
  if ((s = ensure_dt(c)) != CFD_OK) return s;
  const bool check = c->cfg.debug_flags & CFD_CHECK_FINITE;
  const bool graph = c->use_graph && c->exec_mode != CFD_EXEC_PER_BLOCK && !c->profiling && !c->cfg.debug_flags;
  if (graph && !c->graph_valid && nsteps > 0)
    if ((s = build_graph(c)) != CFD_OK) return s;
  for (int n = 0; n < nsteps; ++n) {
    if (check && (s = debug_clear(c)) != CFD_OK) return s;
    if (graph) {
      HIP_TRY(c, hipGraphLaunch(c->graph_exec, c->stream));
    } else if ((s = enqueue_step(c, c->stream, c->profiling)) != CFD_OK) {
      return s;
    }
    if (check) {
      bool bad = false;
      if ((s = debug_flagged(c, &bad)) != CFD_OK) return s;
      if (bad)
        return fail(c, CFD_ERR_NONFINITE,
                    "step %d of %d: a stage produced a non-positive or non-finite density or pressure "
                    "(or a non-finite velocity)",
                    n + 1, nsteps);
    }
  }
  if (dev_dt_last) HIP_TRY(c, launch_copy_dt(c->dptr<double>(c->off_dt), dev_dt_last, c->stream));
  return CFD_OK;
}

extern "C" cfd_status cfd_padded_size(cfd_ctx* c, size_t* count) {
  cfd_status s = need(c, true, false);
  if (s != CFD_OK) return s;
  if (!count) return CFD_ERR_ARG;
  *count = (size_t)c->padded_total;
  return CFD_OK;
}

extern "C" cfd_status cfd_padded_primitives(cfd_ctx* c, double* dev_out) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (!dev_out) return CFD_ERR_ARG;
  if (!c->have_state) return fail(c, CFD_ERR_STATE, "no state set");
  if ((s = fill_ghosts(c, c->stA(), c->stream)) != CFD_OK) return s;
  CellArgs a = cell_args(c);
  a.src = c->stA();
  a.dst = dev_out;
  HIP_TRY(c, launch_export_padded(c->dim, a, c->max_padded, (int)c->blocks.size(), c->stream));
  return CFD_OK;
}

extern "C" cfd_status cfd_set_exec(cfd_ctx* c, int mode, int use_graph) {
  if (!c) return CFD_ERR_ARG;
  if (mode != CFD_EXEC_BATCHED && mode != CFD_EXEC_PER_BLOCK && mode != CFD_EXEC_PERSISTENT)
    return fail(c, CFD_ERR_ARG, "bad exec mode");
  c->exec_mode = mode;
  c->use_graph = use_graph ? 1 : 0;
  release_graph(c);
  return CFD_OK;
}

extern "C" cfd_status cfd_set_ghost_exchange(cfd_ctx* c, int mode) {
  if (!c) return CFD_ERR_ARG;
  if (mode != CFD_GHOSTS_DIRECT && mode != CFD_GHOSTS_PACKED) return fail(c, CFD_ERR_ARG, "bad ghost exchange mode");
  c->ghost_mode = mode;
  release_graph(c);
  return CFD_OK;
}

extern "C" cfd_status cfd_set_variant(cfd_ctx* c, int v) {
  if (!c) return CFD_ERR_ARG;
  if (v < 0 || v >= c->nvariants) return fail(c, CFD_ERR_ARG, "variant %d out of range", v);
  c->variant = v;
  release_graph(c);
  return CFD_OK;
}

extern "C" cfd_status cfd_autotune(cfd_ctx* c, int reps, int* chosen) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (!c->have_state) return fail(c, CFD_ERR_STATE, "no state set");
  if (reps < 1) reps = 1;
  s = stage_prep(c, c->stA(), c->stream);
  if (s != CFD_OK) return s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(c, CFD_ERR_HIP, "hipEventCreate failed");
  }
  const int keep = c->variant;
  int best = keep;
  float best_ms = 1e30f;
  hipError_t he = hipSuccess;
  for (int v = 0; v < c->nvariants && s == CFD_OK && he == hipSuccess; ++v) {
    c->variant = v;
    StageArgs a = stage_args(c);
    a.qin = c->stA();
    a.q0 = c->stA();
    a.qout = c->stB();
    a.mode = MODE_STAGE;
    a.alpha = 0.25;
    a.dtmin = nullptr;
    if ((s = launch_stage_all(c, a, c->stream, false)) != CFD_OK) break;  // warm-up
    if ((he = hipEventRecord(e0, c->stream)) != hipSuccess) break;
    for (int r = 0; r < reps && s == CFD_OK; ++r) s = launch_stage_all(c, a, c->stream, false);
    if (s != CFD_OK) break;
    float ms = 0.f;
    if ((he = hipEventRecord(e1, c->stream)) != hipSuccess || (he = hipEventSynchronize(e1)) != hipSuccess ||
        (he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
      break;
    if (ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s == CFD_OK && he != hipSuccess) s = fail(c, CFD_ERR_HIP, "autotune timing: %s", hipGetErrorString(he));
  c->variant = s == CFD_OK ? best : keep;
  release_graph(c);
  if (chosen) *chosen = best;
  return s;
}

extern "C" cfd_status cfd_profile(cfd_ctx* c, int enable) {
  if (!c) return CFD_ERR_ARG;
  c->profiling = enable != 0;
  c->ev_used = 0;
  c->prof_ms = 0.0;
  c->prof_launches = 0;
  return CFD_OK;
}

extern "C" cfd_status cfd_kernel_time(cfd_ctx* c, double* total_ms, long long* launches) {
  if (!c) return CFD_ERR_ARG;
  double ms = c->prof_ms;
  for (size_t i = 0; i < c->ev_used; ++i) {
    HIP_TRY(c, hipEventSynchronize(c->ev_pool[i].b));
    float t = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&t, c->ev_pool[i].a, c->ev_pool[i].b));
    ms += t;
  }
  c->prof_ms = ms;
  c->ev_used = 0;
  if (total_ms) *total_ms = ms;
  if (launches) *launches = c->prof_launches;
  return CFD_OK;
}

extern "C" cfd_status cfd_query(cfd_ctx* c, int what, long long* value) {
  if (!c || !value) return CFD_ERR_ARG;
  int nv = 0;
  const StageVariant* vars = stage_variants(c->dim, &nv);
  switch (what) {
    case CFD_Q_NBLOCKS: *value = (long long)c->hblocks.size(); return CFD_OK;
    case CFD_Q_NVAR: *value = c->nvar; return CFD_OK;
    case CFD_Q_NVARIANTS: *value = nv; return CFD_OK;
    case CFD_Q_VARIANT: *value = c->variant; return CFD_OK;
    case CFD_Q_TILE_X: *value = vars[c->variant].tx; return CFD_OK;
    case CFD_Q_TILE_Y: *value = vars[c->variant].ty; return CFD_OK;
    default: break;
  }
  if (!c->finalized) return fail(c, CFD_ERR_STATE, "context is not finalized");
  switch (what) {
    case CFD_Q_NCELLS: *value = c->ncells; return CFD_OK;
    case CFD_Q_NTILES: *value = (long long)c->tiles_batched[c->variant].size(); return CFD_OK;
    case CFD_Q_NTRANSFERS: *value = (long long)c->xfers.size(); return CFD_OK;
    case CFD_Q_NPATCHES: *value = (long long)c->patches.size(); return CFD_OK;
    case CFD_Q_NNODES: *value = c->nnodes; return CFD_OK;
    case CFD_Q_EXCHANGE_DOUBLES: *value = c->xbuf_doubles; return CFD_OK;
    case CFD_Q_WORKSPACE_BYTES: *value = (long long)c->ws_bytes; return CFD_OK;
    default: return fail(c, CFD_ERR_ARG, "unknown query %d", what);
  }
}

// ---------------------------------------------------------------------------
// adjoint

extern "C" cfd_status cfd_enable_limiter_freezing(cfd_ctx* c, int enable) {
  if (!c) return CFD_ERR_ARG;
  if (c->finalized) return fail(c, CFD_ERR_STATE, "enable_limiter_freezing after finalize");
  if (enable && c->cfg.limiter == CFD_LIM_NONE) return fail(c, CFD_ERR_ARG, "no limiter to freeze");
  c->freezing = enable != 0;
  return CFD_OK;
}

extern "C" cfd_status cfd_freeze_limiter(cfd_ctx* c, int freeze) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (!c->freezing)
    return fail(c, CFD_ERR_STATE, "limiter freezing not enabled before finalize (cfd_enable_limiter_freezing)");
  if (freeze) {
    if (!c->have_state) return fail(c, CFD_ERR_STATE, "no state set");
    if ((s = fill_ghosts(c, c->stA(), c->stream)) != CFD_OK) return s;
    FreezeArgs a{};
    a.blocks = c->dptr<BlockDev>(c->off_blocks);
    a.q = c->stA();
    a.phi = c->dptr<double>(c->off_phi);
    a.limiter = c->cfg.limiter;
    for (int v = 0; v < MAXV; ++v) a.e2[v] = c->cfg.lim_eps[v] * c->cfg.lim_eps[v];
    HIP_TRY(c, launch_freeze(c->dim, a, c->max_padded, (int)c->blocks.size(), c->stream));
  }
  if (c->frozen != (freeze != 0)) release_graph(c);  // the captured step names the stage kernels
  c->frozen = freeze != 0;
  return CFD_OK;
}

extern "C" cfd_status cfd_enable_adjoint(cfd_ctx* c, int enable) {
  if (!c) return CFD_ERR_ARG;
  if (c->finalized) return fail(c, CFD_ERR_STATE, "enable_adjoint after finalize");
  c->adjoint = enable != 0;
  return CFD_OK;
}

static VjpArgs vjp_args(cfd_ctx* c, const double* q, const double* Rb, double scale, double* out, double* acc) {
  VjpArgs a{};
  a.blocks = c->dptr<BlockDev>(c->off_blocks);
  a.xfers = c->dptr<TransferDev>(c->off_xfers);
  a.patches = c->dptr<PatchDev>(c->off_patches);
  a.npatches = (int)c->patches.size();
  a.q = q;
  a.metric = c->metric();
  a.nodes = c->dptr<double>(c->off_nodes);
  a.Rb = Rb;
  a.facebar = c->dptr<double>(c->off_facebar);
  a.qbar = c->dptr<double>(c->off_qbar);
  a.metricbar = c->dptr<double>(c->off_metricbar);
  a.thetabar = c->dptr<double>(c->off_thetabar);
  a.inflow_part = c->dptr<double>(c->off_part);
  a.part_offset = c->dptr<long long>(c->off_partoff);
  a.facemap = c->dptr<int>(c->off_facemap);
  a.fmap_off = c->dptr<long long>(c->off_fmapoff);
  a.vtiles = c->dptr<TileDev>(c->off_vtiles);
  a.inflow_list = c->dptr<int>(c->off_inflowlist);
  a.ninflow = (int)c->inflow_list.size();
  a.out = out;
  a.acc = acc;
  a.acc_mode = 1;
  a.tile_bc = 0;
  a.scale = scale;
  a.gas = make_gas(c->cfg.gamma);
  a.half_eps = 0.5 * c->cfg.muscl_eps;
  a.kappa = c->cfg.muscl_kappa;
  a.efix = c->cfg.efix;
  a.half_inv_efix = c->cfg.efix > 0.0 ? 0.5 / c->cfg.efix : 0.0;
  for (int v = 0; v < MAXV; ++v) a.e2[v] = c->cfg.lim_eps[v] * c->cfg.lim_eps[v];
  return a;
}

static cfd_status need_adjoint(cfd_ctx* c) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (!c->adjoint) return fail(c, CFD_ERR_STATE, "adjoint not enabled before finalize (cfd_enable_adjoint)");
  if (!c->have_state) return fail(c, CFD_ERR_STATE, "no state set");
  return CFD_OK;
}

// Residual VJP at state buffer q (ghosts filled): out = scale * (dR/dQ)^T Rb,
// acc += the same; scale * dJ/dS, dJ/dOmega, dJ/dtheta accumulate.
// One residual VJP at state q: out = scale (dR/dQ)^T Rb and acc += the parts
// selected by acc_mode (bit 0: that product, bit 1: Rb itself).  Rb must not
// alias out or acc.
static cfd_status vjp_core(cfd_ctx* c, const double* q, const double* Rb, double scale, double* out, double* acc,
                           int acc_mode = 1) {
  const int nb = (int)c->blocks.size();
  VjpArgs a = vjp_args(c, q, Rb, scale, out, acc);
  a.acc_mode = acc_mode;
  hipStream_t s = c->stream;
  if (c->dim == 2) {
    a.tile_bc = 1;
    HIP_TRY(c, launch_vjp_tile2d(c->cfg.limiter, a, (int)c->vtiles.size(), s));
  } else {
    HIP_TRY(c, launch_vjp_face(c->dim, c->cfg.limiter, a, c->max_faces, nb, s));
    HIP_TRY(c, launch_vjp_cell(c->dim, c->cfg.limiter, a, c->max_padded, nb, s));
  }
  if (c->need_bgather) HIP_TRY(c, launch_vjp_boundary_gather(c->dim, a, c->max_face_area, nb, s));
  return CFD_OK;
}

static cfd_status copy_thetabar(cfd_ctx* c, double* dev_BCbar) {
  if (!dev_BCbar || c->nparam == 0) return CFD_OK;
  // dJ/dtheta = sum of the per-position partials accumulated since the reset
  HIP_TRY(c, hipMemsetAsync(c->ws + c->off_thetabar, 0, (size_t)std::max(c->nparam, 1) * MAXV * 8, c->stream));
  VjpArgs a = vjp_args(c, c->stA(), nullptr, 1.0, nullptr, nullptr);
  HIP_TRY(c, launch_vjp_inflow_reduce(c->dim, a, c->stream));
  HIP_TRY(c, hipMemcpy2DAsync(dev_BCbar, c->nvar * 8, c->dptr<double>(c->off_thetabar), MAXV * 8, c->nvar * 8,
                              c->nparam, hipMemcpyDeviceToDevice, c->stream));
  return CFD_OK;
}

static cfd_status node_gradient(cfd_ctx* c, double* dev_Xbar) {
  if (!dev_Xbar) return CFD_OK;
  VjpArgs a = vjp_args(c, c->stA(), nullptr, 1.0, nullptr, nullptr);
  HIP_TRY(c, launch_node_vjp(c->dim, a, dev_Xbar, c->max_nodes, (int)c->blocks.size(), c->stream));
  return CFD_OK;
}

extern "C" cfd_status cfd_adjoint_reset(cfd_ctx* c) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (!c->adjoint) return fail(c, CFD_ERR_STATE, "adjoint not enabled");
  HIP_TRY(c, hipMemsetAsync(c->ws + c->off_metricbar, 0, c->metric_doubles * 8, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->ws + c->off_part, 0, c->part_doubles * 8, c->stream));
  return CFD_OK;
}

extern "C" cfd_status cfd_adjoint_result(cfd_ctx* c, double* dev_Xbar, double* dev_BCbar) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (!c->adjoint) return fail(c, CFD_ERR_STATE, "adjoint not enabled");
  if ((s = node_gradient(c, dev_Xbar)) != CFD_OK) return s;
  return copy_thetabar(c, dev_BCbar);
}

extern "C" cfd_status cfd_residual_vjp(cfd_ctx* c, const double* dev_Rbar, double* dev_Qbar, double* dev_Xbar,
                                       double* dev_BCbar) {
  cfd_status s = need_adjoint(c);
  if (s != CFD_OK) return s;
  if (!dev_Rbar || !dev_Qbar) return CFD_ERR_ARG;
  if ((s = cfd_adjoint_reset(c)) != CFD_OK) return s;
  if ((s = fill_ghosts(c, c->stA(), c->stream)) != CFD_OK) return s;
  if ((s = vjp_core(c, c->stA(), dev_Rbar, 1.0, dev_Qbar, nullptr)) != CFD_OK) return s;
  return cfd_adjoint_result(c, dev_Xbar, dev_BCbar);
}

static cfd_status step_vjp_checks(cfd_ctx* c) {
  cfd_status s = need_adjoint(c);
  if (s != CFD_OK) return s;
  if (c->cfg.rk_scheme != CFD_RK_MSTAGE)
    return fail(c, CFD_ERR_UNSUPPORTED, "the step adjoint covers the M-stage scheme (CFD_RK_MSTAGE)");
  if (c->cfg.dt_mode != CFD_DT_FIXED)
    return fail(c, CFD_ERR_UNSUPPORTED, "the step adjoint needs a fixed time step (CFD_DT_FIXED)");
  if (c->cfg.rk_stages > 4) return fail(c, CFD_ERR_UNSUPPORTED, "the step adjoint keeps at most 4 stage states");
  return CFD_OK;
}

// Reverse sweep of one RK step over ghost-filled stage inputs st[0..M-1]
// (Sec. 2 M-stage scheme: Q^(k) = Q^(0) - dt R(Q^(k-1)) / (M-k+1)).
static cfd_status reverse_step(cfd_ctx* c, const double* const* st, double* dev_Qbar);

extern "C" cfd_status cfd_rk_step_vjp(cfd_ctx* c, double* dev_Qbar) {
  cfd_status s = step_vjp_checks(c);
  if (s != CFD_OK) return s;
  if (!dev_Qbar) return CFD_ERR_ARG;
  const int M = c->cfg.rk_stages;
  double* st[4] = {c->stA(), c->stB(), c->stC(), c->dptr<double>(c->off_stD)};
  // recompute the stage states Q^(1..M-1) of this step from Q^(0) in A
  for (int k = 1; k < M; ++k) {
    if ((s = fill_ghosts(c, st[k - 1], c->stream)) != CFD_OK) return s;
    StageArgs a = stage_args(c);
    a.qin = st[k - 1];
    a.q0 = st[0];
    a.qout = st[k];
    a.mode = MODE_STAGE;
    a.alpha = 1.0 / (double)(M - k + 1);
    a.dtmin = nullptr;
    if ((s = launch_stage_all(c, a, c->stream, false)) != CFD_OK) return s;
  }
  if ((s = fill_ghosts(c, st[M - 1], c->stream)) != CFD_OK) return s;
  const double* cst[4] = {st[0], st[1], st[2], st[3]};
  return reverse_step(c, cst, dev_Qbar);
}

extern "C" cfd_status cfd_rk_step_record(cfd_ctx* c, void* dev_stages) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (!dev_stages) return CFD_ERR_ARG;
  if (c->cfg.rk_scheme != CFD_RK_MSTAGE)
    return fail(c, CFD_ERR_UNSUPPORTED, "stage recording covers the M-stage scheme (CFD_RK_MSTAGE)");
  if (!c->have_state) return fail(c, CFD_ERR_STATE, "no state set");
  if ((s = ensure_dt(c)) != CFD_OK) return s;
  const bool cfl = c->cfg.dt_mode != CFD_DT_FIXED;
  hipStream_t hs = c->stream;
  if (cfl)
    HIP_TRY(c, launch_dt_promote(c->dptr<double>(c->off_dt), c->dptr<unsigned long long>(c->off_dtmin), c->cfg.cfl,
                                 1, nullptr, hs));
  const int M = c->cfg.rk_stages;
  double* slot0 = static_cast<double*>(dev_stages);
  double* A = c->stA();
  // stage_prep: ghost fill, and the viscous residual of the stage input in a
  // Navier-Stokes context, exactly as enqueue_step does
  if ((s = stage_prep(c, A, hs)) != CFD_OK) return s;
  HIP_TRY(c, hipMemcpyAsync(slot0, A, (size_t)c->state_doubles * 8, hipMemcpyDeviceToDevice, hs));
  // the first stage reads the copy, so a single stage can write A itself
  const double* in = slot0;
  for (int k = 1; k <= M; ++k) {
    double* out = (k == M) ? A : slot0 + (size_t)k * c->state_doubles;
    if (k > 1 && (s = stage_prep(c, const_cast<double*>(in), hs)) != CFD_OK) return s;
    StageArgs a = stage_args(c);
    a.qin = in;
    a.q0 = A;
    a.qout = out;
    a.mode = MODE_STAGE;
    a.alpha = 1.0 / (double)(M - k + 1);
    a.dtmin = (k == M && cfl) ? c->dptr<unsigned long long>(c->off_dtmin) : nullptr;
    if ((s = launch_stage_all(c, a, hs, false)) != CFD_OK) return s;
    in = out;
  }
  return CFD_OK;
}

extern "C" cfd_status cfd_rk_step_vjp_recorded(cfd_ctx* c, const void* dev_stages, double* dev_Qbar) {
  cfd_status s = step_vjp_checks(c);
  if (s != CFD_OK) return s;
  if (!dev_Qbar || !dev_stages) return CFD_ERR_ARG;
  const double* slot0 = static_cast<const double*>(dev_stages);
  const double* st[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int k = 0; k < c->cfg.rk_stages; ++k) st[k] = slot0 + (size_t)k * c->state_doubles;
  return reverse_step(c, st, dev_Qbar);
}

static cfd_status reverse_step(cfd_ctx* c, const double* const* st, double* dev_Qbar) {
  cfd_status s = CFD_OK;
  const int M = c->cfg.rk_stages;
  // reverse sweep.  With G_k the cotangent of Q^(k) (G_M = dev_Qbar on entry)
  // and V_k = -dt/(M-k+1) (dR/dQ)^T G_k at Q^(k-1): G_{k-1} = V_k for k > 1, and
  // dJ/dQ^(0) = G_M + ... + G_1 + V_1, accumulated in dev_Qbar.
  double* G = c->dptr<double>(c->off_G);
  double* T = c->dptr<double>(c->off_T);
  const double dt = c->cfg.dt_fixed;
  if (M == 1) {
    const size_t bytes = (size_t)c->nvar * c->ncells * 8;
    HIP_TRY(c, hipMemcpyAsync(G, dev_Qbar, bytes, hipMemcpyDeviceToDevice, c->stream));
    return vjp_core(c, st[0], G, -dt, nullptr, dev_Qbar, 1);
  }
  if ((s = vjp_core(c, st[M - 1], dev_Qbar, -dt, G, nullptr, 0)) != CFD_OK) return s;
  for (int k = M - 1; k >= 1; --k) {
    const double sc = -dt / (double)(M - k + 1);
    if ((s = vjp_core(c, st[k - 1], G, sc, k > 1 ? T : nullptr, dev_Qbar, k > 1 ? 2 : 3)) != CFD_OK) return s;
    std::swap(G, T);
  }
  return CFD_OK;
}

extern "C" cfd_status cfd_objective_wall_pressure(cfd_ctx* c, double* dev_J, double* dev_Qbar) {
  cfd_status s = need_adjoint(c);
  if (s != CFD_OK) return s;
  if (!dev_J) return CFD_ERR_ARG;
  VjpArgs a = vjp_args(c, c->stA(), nullptr, 1.0, dev_Qbar, nullptr);
  HIP_TRY(c, hipMemsetAsync(c->ws + c->off_qbar, 0, c->state_doubles * 8, c->stream));
  for (int f = 0; f < 2 * c->dim; ++f)
    HIP_TRY(c, launch_objective(c->dim, a, c->dptr<ChunkDev>(c->off_objchunks), c->obj_begin[f],
                                c->obj_begin[f + 1] - c->obj_begin[f], c->stream));
  HIP_TRY(c, launch_objective_sum(a, c->dptr<int>(c->off_walllist), (int)c->wall_list.size(), dev_J, c->stream));
  if (dev_Qbar) HIP_TRY(c, launch_vjp_finalize(c->dim, a, c->max_cells, (int)c->blocks.size(), c->stream));
  return CFD_OK;
}

extern "C" cfd_status cfd_uniform_state_vjp(cfd_ctx* c, const double* theta_host, const double* dev_Qbar,
                                            double* dev_thetabar) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (!c->adjoint) return fail(c, CFD_ERR_STATE, "adjoint not enabled");
  if (!theta_host || !dev_Qbar || !dev_thetabar) return CFD_ERR_ARG;
  double th[5] = {0, 0, 0, 0, 0};
  for (int v = 0; v < c->nvar; ++v) th[v] = theta_host[v];
  const int parts = (int)std::min<long long>(cfd_ctx::SUM_PARTS, std::max<long long>(1, c->ncells / 256));
  HIP_TRY(c, launch_uniform_state_vjp(c->dim, dev_Qbar, c->ncells, c->dptr<double>(c->off_sumpart), parts,
                                      dev_thetabar, make_gas(c->cfg.gamma), th, c->stream));
  return CFD_OK;
}

extern "C" cfd_status cfd_state_size(cfd_ctx* c, size_t* bytes) {
  cfd_status s = need(c, true, false);
  if (s != CFD_OK) return s;
  if (!bytes) return CFD_ERR_ARG;
  *bytes = (size_t)c->state_doubles * 8;
  return CFD_OK;
}

extern "C" cfd_status cfd_save_state(cfd_ctx* c, void* dev_dst) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (!dev_dst) return CFD_ERR_ARG;
  HIP_TRY(c, hipMemcpyAsync(dev_dst, c->stA(), (size_t)c->state_doubles * 8, hipMemcpyDeviceToDevice, c->stream));
  return CFD_OK;
}

extern "C" cfd_status cfd_load_state(cfd_ctx* c, const void* dev_src) {
  cfd_status s = need(c, true, true);
  if (s != CFD_OK) return s;
  if (!dev_src) return CFD_ERR_ARG;
  HIP_TRY(c, hipMemcpyAsync(c->stA(), dev_src, (size_t)c->state_doubles * 8, hipMemcpyDeviceToDevice, c->stream));
  c->have_state = true;
  c->dt_valid = false;
  return ensure_dt(c);
}
