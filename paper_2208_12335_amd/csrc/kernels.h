// Launchers of the gfx950 kernels (implemented in kernels.hip), called by the host code.
#pragma once

#include <hip/hip_runtime.h>

#include "aims_internal.h"

namespace aims {

enum { kModeDensity = 0, kModeH = 1, kModeS = 2 };

// Persistent launch: counters[8] (zero at launch) and the number of resident workgroups; a
// null counters pointer selects one workgroup per work item.
struct Queue {
  int* counters = nullptr;
  int workgroups = 0;
};

// Device pointers and scalars of one handle, passed by value to the launchers.
struct DeviceView {
  const BatchDesc* batches;
  const SystemDesc* systems;
  const double4* pts;
  const int32_t* perm;
  const int32_t* batch_atoms;
  const int32_t* batch_acol;
  const int32_t* batch_cols;
  const double* atom_xyz;
  const int32_t* atom_species;
  const int32_t* atom_sys;
  const SpeciesDesc* species;
  const int32_t* shell_l;
  const int32_t* shell_fexp;       // int8 form: per shell, exponent of the density-pass balancing
  const int32_t* fn_fexp;          // int8 form: the same per global basis function
  const double* spline64;
  const float* spline32;
  const int64_t* sys_pt_range;     // [n_sys][2] batch-order point range of each system
  const int64_t* sys_batch_range;  // [n_sys][2] batch range of each system
  RadialGrid rg;
  int n_sys;
};

// Workgroups of a 256-thread kernel resident on the current device at once (cached per kernel),
// and the grid of a tiled launch: one workgroup per item, or (persistent) the resident count
// rounded down to a multiple of the 8 XCDs.
int resident_workgroups(const void* fn);
int tile_grid(int n_items, const Queue& q, const void* fn);

hipError_t launch_fill(double* x, size_t n, double val, hipStream_t st);
hipError_t launch_convert_f32(const double* x, float* y, size_t n, hipStream_t st);

template <typename T>
hipError_t launch_phi_eval(const DeviceView& dv, int b0, int nbatch, int mode, const double* v,
                           T* slab1, T* slab2, hipStream_t st);
hipError_t launch_phi_eval_bf16(const DeviceView& dv, int b0, int nbatch, int mode, const double* v,
                                void* slab1, void* slab2, hipStream_t st);
// nbn: point tile = 32 * nbn points (2..5)
// xout != NULL: store X^T = P_b slab1 into xout (function-major slab); n and the E_T partials
// are formed as well unless n_sorted is NULL.  d_sorted != NULL: also the unweighted kinetic
// density D(p) = sum_j X_pj tphi_j(p) per point (batch order), added atomically.
template <typename T>
hipError_t launch_density(const DeviceView& dv, int nbn, const TileItem* items, int n_items, const T* P,
                          const T* slab1, const T* slab2, double* n_sorted, double* et_batch,
                          hipStream_t st, T* xout = nullptr, Queue q = Queue(),
                          double* d_sorted = nullptr);
hipError_t launch_density_bf16(const DeviceView& dv, int nbn, const TileItem* items, int n_items,
                               const float* P, const void* slab1, const void* slab2, double* n_sorted,
                               double* et_batch, hipStream_t st, float* xout = nullptr, Queue q = Queue());
// gpt != NULL: also the per-point sum over atoms of the same terms (3 doubles per point,
// batch order, added atomically): the gradient of the integrand with respect to the point.
template <typename T>
hipError_t launch_pulay(const DeviceView& dv, int b0, int nbatch, const double* v, const T* X,
                        const T* Y, const double* gE, double* dE_dR, hipStream_t st,
                        double* gpt = nullptr);
// Moving-grid terms: the nuclear model potential on the grid (caller order) and the
// partition-weight, potential and point-motion terms of the total gradient.
hipError_t launch_vext(const DeviceView& dv, int64_t n, const int32_t* pt_sys,
                       const int32_t* sys_natoms, const double* atom_Z, const double* sys_model,
                       double* v_out, hipStream_t st);
hipError_t launch_gridforce(const DeviceView& dv, int nbatch, int max_sys_atoms,
                            const int32_t* sys_natoms, const double* atom_Z, const double* sys_model,
                            const int32_t* pt_owner, const double* pt_wgrid, const double* v_model,
                            const double* n_sorted, const double* d_sorted, const double* gpt,
                            const double* gE, double* dE_dR, hipStream_t st);
// Wave-per-point form for systems of at most 64 k_chunks atoms (k_chunks in 1, 2, 4, 8):
// `ranges` are runs of consecutive batches of one system, each with its slot of 3 n_a doubles in
// `part` (the slots of system s start at sys_part_off[s], sys_nrange[s] of them); a second kernel
// adds them, in slot order, times gE into dE_dR.
struct ForceRange {
  int32_t b0, b1;     // batches [b0, b1)
  int32_t sys;
  int32_t pad;
  int64_t part_off;   // element offset of this range's slot in `part`
};
hipError_t launch_gridforce_wave(const DeviceView& dv, int k_chunks, const ForceRange* ranges,
                                 int n_ranges, int max_sys_atoms, const int32_t* sys_natoms,
                                 const double* atom_Z, const double* sys_model,
                                 const int64_t* sys_pair_off, const double* inv_aR,
                                 const int32_t* pt_owner, const double* v_model,
                                 const double* n_sorted, const double* d_sorted, const double* gpt,
                                 double* part, const int64_t* sys_part_off, const int32_t* sys_nrange,
                                 const double* gE, double* dE_dR, hipStream_t st);
hipError_t launch_scale(double* y, const double* x, size_t n, const double* gE, hipStream_t st);
hipError_t launch_dv(const DeviceView& dv, double* dE_dv, const double* n_sorted, int64_t n,
                     const double* gE, hipStream_t st);
template <typename T>
hipError_t launch_hs(const DeviceView& dv, const TileItem* items, int n_items, const T* slab1,
                     const T* slab2, double* out, hipStream_t st, Queue q = Queue(), int te = 64);
hipError_t launch_hs_bf16(const DeviceView& dv, const TileItem* items, int n_items, const void* slab1,
                          const void* slab2, double* out, hipStream_t st, Queue q = Queue());
hipError_t launch_zero_int(int* x, int n, hipStream_t st);
// Positions given on the device: flag = 1 if any atom is not finite or farther than margin from
// xyz0; the outputs of such a call are then set to NaN (launch_poison, a no-op when flag = 0).
hipError_t launch_positions_check(const double* xyz, const double* xyz0, int n, double margin,
                                  int* flag, hipStream_t st);
hipError_t launch_poison(double* x, size_t n, const int* flag, hipStream_t st);
// Sliced integer form (int8.hip): P as digit words with one exponent per row; basis slabs of
// digit words with per-point (density) or per-column (H, S) exponents; the tiled int8 kernels.
hipError_t launch_slice_p(const DeviceView& dv, const double* P, uint64_t* P8, int32_t* eP,
                          int64_t n_rows, hipStream_t st);
hipError_t launch_phi_eval_i8(const DeviceView& dv, int b0, int nbatch, int mode, const double* v,
                              uint64_t* slab1, uint64_t* slab2, int32_t* ex1, int32_t* ex2,
                              int max_slots, hipStream_t st);
hipError_t launch_density_i8(const DeviceView& dv, const TileItem* items, int n_items,
                             const uint64_t* P8, const int32_t* eP, const uint64_t* slab1,
                             const uint64_t* slab2, const int32_t* ex1, const int32_t* ex2,
                             double* n_sorted, double* et_batch, hipStream_t st, Queue q = Queue());
hipError_t launch_hs_i8(const DeviceView& dv, const TileItem* items, int n_items, const uint64_t* slab1,
                        const uint64_t* slab2, const int32_t* ex1, const int32_t* ex2, double* out,
                        hipStream_t st, Queue q = Queue());
hipError_t prepare_launch_configs_i8();
hipError_t prepare_launch_configs();
hipError_t launch_density_finish(const DeviceView& dv, const double* n_sorted, const double* v,
                                 double* n_out, double* part, int nblk, const double* et_batch,
                                 double* sums_out, hipStream_t st);

}  // namespace aims
