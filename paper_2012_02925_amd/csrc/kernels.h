// Launch interface between the host planner (api.hip) and the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "cfd_internal.h"
#include "device_math.h"

namespace cfd {

struct StageArgs;  // stage_kernel.h

struct GhostArgs {
  const BlockDev* blocks;
  const TransferDev* xfers;
  const PatchDev* patches;
  const ChunkDev* chunks;
  int chunk_begin;
  double* q;              // state buffer whose ghosts are filled
  double* buf;            // exchange buffer
  const double* bcparams;  // boundary parameters, MAXV doubles per parameter slot
  const double* metric;
  Gas gas;
  // non-null: the first wavefront of workgroup 0 also forms the time step,
  // dt <- cfl * min over the DT_SLOTS slots, slots <- +inf (the promote of a
  // step folded into its first ghost launch)
  double* dt;
  unsigned long long* dtmin;
  double cfl;
};

struct CellArgs {
  const BlockDev* blocks;
  const double* src;
  double* dst;
  const double* metric;
  const long long* offsets;  // export_padded: output offset per block
  unsigned long long* dtmin;
  double* dtloc;  // non-null: also write cfl * Omega/lambda per cell (packed)
  double cfl;
  int* err;
  int flag_primitive;
  Gas gas;
  double visc_cv;  // viscous time-step coefficient (0: inviscid)
};

// Classical fourth-order Runge-Kutta combination (primitive padded states).
struct Rk4Args {
  const BlockDev* blocks;
  const double* q;   // step input Q
  const double* y2;  // Q - dt/2 R(Q)
  const double* y3;  // Q - dt/2 R(Y2)
  const double* y4;  // Q - dt R(Y3)
  const double* z;   // Q - dt/6 R(Y4)
  double* out;       // Q^(n+1) (may be q)
  Gas gas;
};

struct MetricArgs {
  const BlockDev* blocks;
  const double* nodes;
  double* metric;
  int* err;
};

struct StageVariant {
  int tx, ty, kc;
};

const StageVariant* stage_variants(int dim, int* count);
hipError_t launch_sumsq(int nvar, const double* R, long long ncells, double* partial, int nparts,
                        double* norms, hipStream_t s);
// ff: some block has a farfield patch (selects the kernels that test for it);
// persistent: cap the grid at the workgroups the device holds at once (the
// kernel's grid-stride loop then walks the rest of the tile list)
hipError_t launch_stage(int dim, int flux, int lim, int variant, bool ff, const StageArgs& a, int grid,
                        bool persistent, hipStream_t s);
hipError_t launch_ghost(int dim, const GhostArgs& a, int nchunks, hipStream_t s);
hipError_t launch_set_state(int dim, const CellArgs& a, long long max_cells, int nblocks, hipStream_t s);
hipError_t launch_get_state(int dim, const CellArgs& a, long long max_cells, int nblocks, hipStream_t s);
hipError_t launch_cell_dt(int dim, const CellArgs& a, long long max_cells, int nblocks, hipStream_t s);

// Limiter freezing: frozen factors of every cell -1 .. n per direction from a
// ghost-filled primitive state (0 elsewhere in the padded arrays).
struct FreezeArgs {
  const BlockDev* blocks;
  const double* q;  // primitive state buffer, ghosts filled
  double* phi;      // frozen-limiter buffer: per block dim * nvar padded arrays
  int limiter;      // LIM_VANLEER or LIM_VANALBADA
  double e2[MAXV];
};
hipError_t launch_freeze(int dim, const FreezeArgs& a, long long max_padded, int nblocks, hipStream_t s);
hipError_t launch_export_padded(int dim, const CellArgs& a, long long max_padded, int nblocks, hipStream_t s);
hipError_t launch_metrics(int dim, const MetricArgs& a, long long max_pos, int nblocks, hipStream_t s);
hipError_t launch_dt_promote(double* dt, unsigned long long* dtmin, double cfl, int promote, double* out,
                             hipStream_t s);
hipError_t launch_set_u64(unsigned long long* p, unsigned long long v, int n, hipStream_t s);
// debug checks: NaN into the ghost region of a state buffer (a.dst); flag
// (a.err) a non-physical interior cell of a primitive buffer (a.src); flag a
// non-finite entry of a packed array
hipError_t launch_nan_ghosts(int dim, const CellArgs& a, long long max_padded, int nblocks, hipStream_t s);
hipError_t launch_check_state(int dim, const CellArgs& a, long long max_cells, int nblocks, hipStream_t s);
hipError_t launch_rk4_combine(int dim, const Rk4Args& a, long long max_cells, int nblocks, hipStream_t s);
hipError_t launch_check_packed(const double* x, long long n, int* err, hipStream_t s);
hipError_t launch_copy_dt(const double* src, double* dst, hipStream_t s);

}  // namespace cfd
