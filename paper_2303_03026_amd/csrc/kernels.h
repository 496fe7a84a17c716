// Launch interface between the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device_mhd.h"

namespace amrvac {

// Face link kinds of the neighbour table (one record per block face).
enum { LINK_SAME = 0, LINK_FINE = 1, LINK_COARSE = 2, LINK_PHYS = 3 };
constexpr int LINK_INTS = 6;  // kind, id[4] (or bc kind in id[0]), unused
constexpr int MAXLEV = 12;

// Block shape of a context, by value in kernel arguments.
struct GridConst {
  int ndim;
  int nx;
  int ng;
  int pn;       // nx + 2 ng
  int nb;       // blocks of the plain path's scratch (single-job contexts)
  int nfaces;   // faces per block per direction: (nx+1) nx^(ndim-1)
  long pcells;  // padded cells per block
  long icells;  // interior cells per block
  int precision;
};

// Per-block tables of the block pool (indexed by pool block id) plus the
// active block list in execution order.
struct Tables {
  const int* level;      // [cap] 1-based level
  const int* job;        // [cap] job slot
  const double* inv_dx;  // [cap][3] 1/dx of the block's level
  const int* link;       // [cap][6][LINK_INTS]
  const int* pos;        // [cap][3] block position on its level
  const int* wrap;       // [cap][3] cells per direction on the block's level
  const int* order;      // [nactive] active blocks, Morton order within each job
  int nactive;
};

// Per-job time-step scalars, indexed by job slot; a stage advances by
// dt_scale * dt (1 for SSPRK(2,2)/(3,3), 1/2 for the SSPRK(4,3) stages, the
// beta/alpha ratios of the SSPRK(5,4) stages).
struct JobScalars {
  const double* dt;
  const double* ch;
  const double* kappa;
  double dt_scale = 1.0;
};

// Per-job CFL state: running max rate (non-negative double bits), NaN mark,
// geometry (sum_d 1/dx_d and min_d dx_d on the job's finest level, Courant
// number, psi damping coefficient; cfl == 0 marks an unused slot) and the
// outputs.
struct JobCfl {
  unsigned long long* rate_bits;
  unsigned int* nan;
  const double* geom;  // [njobs][4]
  double* dt;
  double* ch;
  double* kappa;
  int njobs;
  // nonzero: the cells next to faces towards finer leaves are left out of
  // the folded rate (the coarse/fine flux correction changes them after the
  // stage; launch_cfl_reflux_cells folds them in afterwards)
  int skip_fine = 0;
};

struct FixedBC {
  double prim[3][2][NV];
};

// ghost filling ------------------------------------------------------------
// tasks: (block, face) pairs; one list for copy/restrict/physical faces and
// one for prolongation (run after the first)
hipError_t launch_fill_faces(hipStream_t s, const GridConst& G, const int* tasks, int ntasks, const Tables& T,
                             void* slot, const PhysConst& P, const FixedBC& fixed);
// The faces towards coarser leaves (prolongation tasks) only, one thread per
// fine ghost layer and coarse cell across the face; results equal those of
// launch_fill_faces on the same tasks.
hipError_t launch_prolong_faces(hipStream_t s, const GridConst& G, const int* tasks, int ntasks, const Tables& T,
                                void* slot);

// plain stage (single-job FP64 contexts; scalars are element 0) -------------
hipError_t launch_prim(hipStream_t s, const GridConst& G, const void* slot, double* prim, const PhysConst& P,
                       DevStatus* st);
hipError_t launch_flux(hipStream_t s, const GridConst& G, int dir, const double* prim, double* flux,
                       const double* ch_dev, const PhysConst& P, const double* inv_dx);
struct FluxPtrs {
  double* f[3];
};
hipError_t launch_reflux(hipStream_t s, const GridConst& G, const int* tasks, int ntasks, const Tables& T,
                         FluxPtrs flux);
hipError_t launch_update(hipStream_t s, const GridConst& G, const Tables& T, const void* in, const void* base,
                         void* out, double w, FluxPtrs flux, const double* dt_dev, double dt_scale,
                         const double* kappa_dev);

// fused stage (nx = 16) and the coarse/fine correction that follows it -------
// Launch shape of the fused stage (results do not depend on it):
//   zseg: workgroups per block, each marching BN / zseg z planes (1, 2, 4;
//         3D only)
//   rot:  rotate the per-plane extra work (halo cells, halo slopes, 17th
//         faces) over the four waves of a workgroup
//   xcd:  give each XCD a contiguous run of the block list
struct FusedTune {
  int zseg;
  int rot;
  int xcd;
};
// cfl (may be null): also fold each job's CFL rate of the output interior
// into cfl->rate_bits / cfl->nan (as launch_cfl_accumulate would from out).
// The fused stage of blocks with three ghost layers (the five-cell
// reconstructions), FP64 or FP32-mixed.  part: 3D only, nb x NV x nx^3
// doubles of scratch for the in-plane flux differences.  freg and cfl (may
// be null): flux registers and CFL folding as for launch_fused_stage.
hipError_t launch_fused5_stage(hipStream_t s, const GridConst& G, const Tables& T, const JobScalars& J, const void* in,
                               const void* base, void* out, double w, const PhysConst& P, DevStatus* st,
                               double* part, void* freg, const JobCfl* cfl);
// freg (may be null): flux registers, [cap][6 faces][NV][face cells] in the
// face precision (face cells nx^2 in 3D, nx in 2D, transverse index t1 + nx
// t2 with t1 along the face's first transverse axis: y for x faces, x
// otherwise).  The stage stores there the face fluxes it evaluates on block
// faces towards finer or coarser leaves.
hipError_t launch_fused_stage(hipStream_t s, const GridConst& G, const Tables& T, const JobScalars& J,
                              const FusedTune& tune, const void* in, const void* base, void* out, double w,
                              const PhysConst& P, DevStatus* st, const JobCfl* cfl, void* freg);
// Coarse/fine flux correction of out from the flux registers freg that the
// fused stage filled.  tasks: (block, face) pairs grouped by direction;
// direction d's are pairs first[d] .. first[d] + count[d] - 1 (host arrays).
// hipErrorInvalidValue if there are tasks and freg is null.
hipError_t launch_reflux_apply(hipStream_t s, const GridConst& G, const Tables& T, const JobScalars& J,
                               const int* tasks, const int first[3], const int count[3], void* out, double w,
                               const void* freg);
// After the correction of a stage that folded its CFL rate with
// C.skip_fine: fold in the rates of the corrected cells (the coarse cells
// next to each task's face).
hipError_t launch_cfl_reflux_cells(hipStream_t s, const GridConst& G, const Tables& T, const int* tasks,
                                   int ntasks, const void* slot, const PhysConst& P, DevStatus* st,
                                   const JobCfl& C);

// regrid transfer tasks: kind, new block, up to 8 sources (see k_regrid)
enum { REGRID_COPY = 0, REGRID_PROLONG = 1, REGRID_RESTRICT = 2 };
constexpr int REGRID_TASK_INTS = 10;
hipError_t launch_regrid(hipStream_t s, const GridConst& G, const Tables& Told, const int* tasks, int ntasks,
                         const void* old_slot, void* new_slot);

// out = a + coef (b - a) on the leaf interior cells of the active blocks
// Loehner indicator parameters: per-variable weights of the conserved
// variables and the wave filter epsilon.
struct LohnerParams {
  double weight[NV];
  double wavefilter;
};

hipError_t launch_lohner(hipStream_t s, const GridConst& G, const Tables& T, const void* slot, const LohnerParams& L,
                         double* ind);
hipError_t launch_combine(hipStream_t s, const GridConst& G, const Tables& T, const void* a, const void* b,
                          double coef, void* out);

// CFL: per-job max rate over the active blocks (accumulate), then per-job
// dt, c_h, kappa, which also empties the accumulators (finalize); launch_cfl
// does both.  launch_cfl_clear empties the accumulators.
hipError_t launch_cfl_accumulate(hipStream_t s, const GridConst& G, const Tables& T, const void* slot,
                                 const PhysConst& P, DevStatus* st, const JobCfl& C);
hipError_t launch_cfl_finalize(hipStream_t s, DevStatus* st, const JobCfl& C);
hipError_t launch_cfl(hipStream_t s, const GridConst& G, const Tables& T, const void* slot, const PhysConst& P,
                      DevStatus* st, const JobCfl& C);
hipError_t launch_cfl_clear(hipStream_t s, const JobCfl& C);

// conversion over the block range [first, first + count) ------------------
hipError_t launch_set_prim(hipStream_t s, const GridConst& G, int first, int count, const double* prim, void* slot,
                           const PhysConst& P);
hipError_t launch_get_cons(hipStream_t s, const GridConst& G, int first, int count, const void* slot,
                           double* cons);
hipError_t launch_reset_status(hipStream_t s, DevStatus* st);

}  // namespace amrvac
