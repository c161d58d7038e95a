// Internal data layout shared by the host set-up code and the gfx950 kernels.
//
// Device-resident state of one handle (all in HBM, uploaded once at set-up):
//   pts[n]        double4 (x, y, z, w) of every point, in batch order
//   perm[n]       caller index of each batch-ordered point
//   batches[nB]   BatchDesc, in the spatial order produced by the bisection
//   batch_atoms   per batch: global atom index of each relevant atom
//   batch_acol    per batch: first batch-local basis column of each relevant atom
//   batch_cols    per batch: system basis index of each batch-local column
//   atom_xyz      double [n_atoms][3] positions used by the next call
//   atom_species  int    [n_atoms] global species index
//   species       SpeciesDesc per species; spline64 / spline32 coefficient tables
//   scratch       two slabs (Phi^T and a second operand) for one group of batches
#pragma once

#include <cstdint>

namespace aims {

constexpr int kLmax = 3;
constexpr int kMaxShells = 32;      // shells per species
constexpr int kMaxBatch = 512;      // points per batch
constexpr int kTile = 64;           // output tile edge of the MFMA kernels
constexpr int kPad = 32;            // slab rows are padded to a multiple of this many points
constexpr int kMaxBasis = 65535;    // basis functions per system (32-bit offsets into P)

struct BatchDesc {
  int32_t pt_off;     // first point (batch order)
  int32_t n_p;        // points
  int32_t atom_off;   // into batch_atoms / batch_acol
  int32_t n_atoms;    // relevant atoms
  int32_t col_off;    // into batch_cols
  int32_t n_b;        // nonzero basis functions
  int32_t sys;        // system index
  int32_t ldp;        // slab row length: n_p rounded up to kPad
  int64_t slab_off;   // element offset of this batch's slab rows inside the group scratch
};

struct SpeciesDesc {
  int32_t nshell;
  int32_t nfn;
  int32_t lmax;
  int32_t shell_l_off;   // into the device shell_l table
  int64_t spline_off;    // element offset: coefficients at [(k * nshell + j) * 8 + c]
};

struct SystemDesc {
  int64_t mat_off;       // element offset of this system's nb x nb matrices
  int32_t nb;            // basis size (leading dimension)
  int32_t atom_off;      // first global atom of the system
  int64_t row_off;       // first global basis row of the system (sum of the earlier nb)
};

struct RadialGrid {      // shared by all systems of a handle
  double s0;             // ln r0
  double h;              // knot spacing in ln r
  double inv_h;
  double rc;
  int32_t n_log;
};

// Work item of the tiled MFMA kernels: one output tile of one batch.
struct TileItem {
  int32_t batch;         // global batch index
  int16_t ti, tj;        // tile row / column
};

}  // namespace aims
