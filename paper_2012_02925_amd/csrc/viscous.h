// Laminar viscous terms (Sec. 2, eq. (governing): F_v,n = (0, tau . n,
// Theta . n), face gradients by Green's theorem on a wider stencil).
//
// Geometry (once per grid): cell centres (mean of the cell's nodes) in padded
// arrays with the first ghost layer filled (across a connection the donor's
// centre moved by the offset between the two face centres; at a physical
// boundary the interior centre mirrored in the boundary face's plane), and
// pseudo-node positions (mean centre of the interior and face-ghost cells
// around each grid node).  Per stage: pseudo-node values of (u.., T) with
// T = gamma p / rho, then once per face the Green's-theorem gradient over the
// face's dual volume (the two cell centres and the face's pseudo-nodes), the
// Stokes stresses, Theta = u . tau + k grad T and F_v . S, and per cell
// Rv = (1/Omega) sum F_v . S_out, which the stage kernel subtracts from the
// inviscid residual.
#pragma once

#include <hip/hip_runtime.h>

#include "cfd_internal.h"

namespace cfd {

struct ViscArgs {
  const BlockDev* blocks;
  const TransferDev* xfers;
  const PatchDev* patches;
  const ChunkDev* chunks;  // ghost-fill chunk list 1 (transfer packs and physical patches)
  const double* nodes;     // grid nodes [coord][node]
  const double* metric;
  double* centers;         // padded arrays from BlockDev::corigin: dim cell-centre coordinates
  double* npos;            // pseudo-node positions [coord][node]
  const double* q;         // primitive state buffer, face ghosts filled
  double* rv;              // viscous residual [(momentum.., energy)][cell], packed
  double mu;               // viscosity
  double kcond;            // conductivity mu / ((gamma - 1) Pr)
  double gamma;
  const TileDev* tiles;    // tiles of viscous_tile_shape over every block (fused pass)
  int ntiles;
  int wrap;                // read the state of periodic neighbours through the wrap (BlockDev::wrap)
};

// Tile shape (cells along i, j and planes along k) of the fused pass; the
// host lists tiles of this shape over every block.
void viscous_tile_shape(int dim, int* tx, int* ty, int* tk);

hipError_t launch_cell_centers(int dim, const ViscArgs& a, long long max_cells, int nblocks, hipStream_t s);
hipError_t launch_ghost_centers(int dim, const ViscArgs& a, int nchunks, hipStream_t s);
// pseudo-node positions from the centres (set-up); max_nodes bounds the node
// count of a block
hipError_t launch_pseudo_nodes(int dim, const ViscArgs& a, long long max_nodes, int nblocks, hipStream_t s);
// Per stage: one fused tiled pass over the tile list (2D or 3D); the pass
// stages the pseudo-node values of (u.., T) of each tile in LDS itself.
hipError_t launch_viscous(int dim, const ViscArgs& a, hipStream_t s);

}  // namespace cfd
