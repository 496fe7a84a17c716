// Launch interface between the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device_mhd.h"

namespace amrvac {

// Face link kinds of the neighbour table (one record per block face).
enum { LINK_SAME = 0, LINK_FINE = 1, LINK_COARSE = 2, LINK_PHYS = 3 };
constexpr int LINK_INTS = 6;  // kind, id[4] (or bc kind in id[0]), unused

// Geometry of the block set, by value in kernel arguments.
struct GridConst {
  int ndim;
  int nx;
  int ng;
  int pn;       // nx + 2 ng
  int nb;
  int nfaces;   // faces per block per direction: (nx+1) nx^(ndim-1)
  long pcells;  // padded cells per block
  long icells;  // interior cells per block
  int base[3];
  int precision;
};

// Per-level spacing (levels 1..MAXLEV), by value.
constexpr int MAXLEV = 12;
struct LevelConst {
  double dx[MAXLEV + 1][3];
  double inv_dx[MAXLEV + 1][3];
  double sum_inv_dx_fin;  // sum_d 1/dx_d on the finest leaf level
  double min_dx_fin;      // min_d dx_d on the finest leaf level
  double cfl;
  double glm_alpha;
};

struct FixedBC {
  double prim[3][2][NV];
};

// ghost filling ------------------------------------------------------------
// tasks: (block, face) pairs; phase 0 = copy/restrict/physical, 1 = prolong
hipError_t launch_fill_faces(hipStream_t s, const GridConst& G, const int* tasks, int ntasks,
                             const int* link, const int* pos, void* slot, const PhysConst& P,
                             const FixedBC& fixed);

// plain stage --------------------------------------------------------------
hipError_t launch_prim(hipStream_t s, const GridConst& G, const void* slot, double* prim,
                       const PhysConst& P, DevStatus* st);
hipError_t launch_flux(hipStream_t s, const GridConst& G, int dir, const double* prim, double* flux,
                       const double* ch_dev, const PhysConst& P);
struct FluxPtrs {
  double* f[3];
};
hipError_t launch_reflux(hipStream_t s, const GridConst& G, const int* tasks, int ntasks,
                         const int* link, FluxPtrs flux);
hipError_t launch_update(hipStream_t s, const GridConst& G, const LevelConst& L, const int* level,
                         const void* in, const void* base, void* out, double w,
                         FluxPtrs flux, const double* dt_dev, const double* kappa_dev);

// fused stage (FP64, nx = 16) and the coarse/fine correction that follows it
hipError_t launch_fused_stage(hipStream_t s, const GridConst& G, const LevelConst& L, const int* level,
                              const int* link, const int* order, const void* in, const void* base, void* out,
                              double w, const double* dt_dev, const double* ch_dev, const double* kappa_dev,
                              const PhysConst& P, DevStatus* st);
hipError_t launch_reflux_correct(hipStream_t s, const GridConst& G, const LevelConst& L, const int* level,
                                 const int* tasks, int ntasks, const int* link, const void* in, void* out, double w,
                                 const double* dt_dev, const double* ch_dev, const PhysConst& P);

// CFL ----------------------------------------------------------------------
hipError_t launch_cfl(hipStream_t s, const GridConst& G, const LevelConst& L, const int* level,
                      const void* slot, const PhysConst& P, DevStatus* st, double* dt_dev,
                      double* ch_dev, double* kappa_dev);

// conversion -----------------------------------------------------------------
hipError_t launch_set_prim(hipStream_t s, const GridConst& G, const double* prim, void* slot,
                           const PhysConst& P);
hipError_t launch_get_cons(hipStream_t s, const GridConst& G, const void* slot, double* cons);
hipError_t launch_reset_status(hipStream_t s, DevStatus* st);

}  // namespace amrvac
