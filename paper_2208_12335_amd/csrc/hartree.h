// Hartree potential by atom-centred multipole expansion (hartree.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace aims {

constexpr int kHartreeBlocks = 256;   // blocks per system of the potential kernel
constexpr int kHartreeMaxL = 6;
constexpr int kGauss = 6;             // Gauss-Legendre points per radial interval

struct HartreeShell {       // the points of one radial node of one atom
  int32_t atom;             // global atom index
  int32_t p0, p1;           // range in shell_pts (batch-order point indices)
  int32_t out;              // atom * K_max + node
  double inv_w;             // 1 / W_node (radial weight with r^2)
};

struct HartreeSys {         // the radial grid of one system
  int32_t K;                // radial nodes
  int32_t K_max;            // node stride of the per-atom arrays (largest K of the handle)
  int32_t fac_off;          // offset of this K's spline factors in cp / den
  int32_t pad;
  double r_map;             // Becke map: r = r_map cot^2(theta/2), theta_k = (k+1) pi/(K+1)
};

struct HartreeDev {
  int l_max = 0;
  int n_atoms = 0;
  int n_shells = 0;
  const HartreeShell* shells = nullptr;
  const int32_t* shell_pts = nullptr;
  const HartreeSys* sys = nullptr;          // [n_sys]
  const int32_t* sys_natoms = nullptr;
  const int32_t* edge = nullptr;            // [n_atoms]: edge node (splines over edge..K-1)
  const double* r_edge = nullptr;           // [n_atoms]: its radius (exterior form from there on)
  const double* cp = nullptr;               // Thomas factors of the natural-spline system
  const double* den = nullptr;
  const double* gl = nullptr;               // [2 kGauss]: nodes on [-1, 1], then weights
  double* rho = nullptr;                    // [n_atoms][K_max][(l_max+1)^2]
  double* Mr = nullptr;
  double* V = nullptr;
  double* MV = nullptr;
  double* q = nullptr;                      // [n_atoms][(l_max+1)^2]
  double4* Vc = nullptr;                    // [n_atoms][K_max][(l_max+1)^2] cubic coefficients
  double* part = nullptr;                   // [n_sys][kHartreeBlocks]
};

// v_out (caller order) = v_H of the density n (caller order); E_or_null[s] = 1/2 sum w n v_H
hipError_t launch_hartree(const DeviceView& dv, const HartreeDev& hd, const double* n,
                          double* v_out, double* E_or_null, hipStream_t st);

}  // namespace aims
