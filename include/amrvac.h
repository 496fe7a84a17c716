/*
 * amrvac.h - C ABI of the MI355X (gfx950) explicit GLM-MHD block-AMR hot path.
 *
 * The library advances the ideal MHD equations with GLM divergence cleaning
 * on a static block-based quadtree/octree hierarchy (refinement ratio 2,
 * leaf blocks of block_nx^ndim cells with nghost ghost layers), as described
 * in MPI-AMRVAC 3.0 (arXiv 2303.03026): conservative finite volumes inside
 * SSP Runge-Kutta steps ("Schemes and limiters for HD and MHD", Table
 * tab:schemes_time), van Leer limited reconstruction of primitive variables
 * with 2 ghost cells (Table t:limiters), HLL fluxes (Table tab:schemes_space)
 * and the 'glm' monopole control (Table t:divb).
 *
 * Conventions used by every call
 *   - Variables, in this order: rho, m_x, m_y, m_z, e, B_x, B_y, B_z, psi
 *     (conserved) and rho, v_x, v_y, v_z, p, B_x, B_y, B_z, psi (primitive);
 *     magnetic pressure |B|^2/2.  2D runs keep all three vector components.
 *   - State slots are device buffers OWNED BY THE CALLER (e.g. torch tensors),
 *     registered once in amrvac_init_blocks, never freed by the library.
 *     Layout is block-major: slot = [block][var][cell] with padded blocks of
 *     pn^ndim cells, pn = block_nx + 2*nghost, cell index
 *     ((k+ng)*pn + (j+ng))*pn + (i+ng) (3D; 2D drops k), i fastest.
 *       AMRVAC_FP64:       9 arrays of double per block (72 B per cell).
 *       AMRVAC_FP32_MIXED: 8 float arrays (rho, m_x, m_y, m_z, B_x, B_y, B_z,
 *                          psi) followed by one double array (e) per block
 *                          (40 B per cell).
 *     An FP64 slot's blocks start AMRVAC_SLOT_LEAD_FP64 bytes into the
 *     buffer, so that with a 32-byte aligned buffer every interior row
 *     (i = 0 .. block_nx-1) begins on a 32-byte memory sector; FP32-mixed
 *     slots start at byte 0.  amrvac_slot_bytes gives the size, lead
 *     included.  Only face ghost slabs are used; edge and corner cells of
 *     the padded block are never read or written.
 *   - Every call enqueues work on the stream given at init (a hipStream_t,
 *     caller-owned) and returns without synchronising, except
 *     amrvac_sync_flags and amrvac_destroy.
 *   - Every call returns AMRVAC_OK (0) or a negative status; the context keeps
 *     a message (amrvac_last_error).  HIP errors keep their hipError_t text.
 *   - Calls on one context are not thread-safe.
 */
#ifndef AMRVAC_H
#define AMRVAC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amrvac_ctx amrvac_ctx;

enum amrvac_status {
  AMRVAC_OK = 0,
  AMRVAC_E_ARG = -1,          /* invalid argument or block table            */
  AMRVAC_E_HIP = -2,          /* a HIP runtime call failed                  */
  AMRVAC_E_NOMEM = -3,        /* library-owned device memory unavailable    */
  AMRVAC_E_NONPHYSICAL = -4,  /* small density/pressure or invalid dt seen  */
  AMRVAC_E_STATE = -5         /* call not valid in the context's state      */
};

enum { AMRVAC_FP64 = 0, AMRVAC_FP32_MIXED = 1 };
enum { AMRVAC_BC_PERIODIC = 0, AMRVAC_BC_ZEROGRAD = 1, AMRVAC_BC_REFLECT = 2, AMRVAC_BC_FIXED = 3 };
enum { AMRVAC_FLAG_SMALL_RHO = 1, AMRVAC_FLAG_SMALL_P = 2, AMRVAC_FLAG_BAD_DT = 4 };
enum { AMRVAC_PATH_PLAIN = 0, AMRVAC_PATH_FUSED = 1 };
/* Reconstruction limiters (Table t:limiters; all on the 2-ghost-cell
 * stencil): 'vanleer' (van Leer 1974, the harmonic slope), 'koren' (Koren
 * 1993) and 'cada3' (Cada and Torrilhon 2009, their third-order limiter
 * function without the smooth-extremum switch).  With d- and d+ the backward
 * and forward differences of a primitive variable, a cell's right and left
 * face values are w + phi d+ / 2 and w - phi' d- / 2; koren and cada3 give
 * the unlimited third-order values (2 d+ + d-)/6 and (2 d- + d+)/6 in smooth
 * monotone regions. */
enum { AMRVAC_LIM_VANLEER = 0, AMRVAC_LIM_KOREN = 1, AMRVAC_LIM_CADA3 = 2, AMRVAC_LIM_WENO5 = 3, AMRVAC_LIM_WENOZ5 = 4,
       AMRVAC_LIM_MP5 = 5, AMRVAC_LIM_WENOZP5 = 6 };
/* The fifth-order reconstructions of Table t:limiters on 3 ghost cells
 * (nghost = 3; FP64 on the per-kernel and the fused path, FP32-mixed on
 * the fused path with the nonlinear weights in FP64), each face value from the five
 * cells on its side: 'weno5' (Jiang and Shu 1996, eps = 1e-6), 'wenoz5'
 * (Borges et al. 2008, WENO-Z weights, eps = 1e-40), 'wenozp5' (Acker et al.
 * 2016, WENO-Z+ weights with lambda = dx^(2/3) of the block, eps = 1e-40) and
 * 'mp5' (Suresh and Huynh 1997, monotonicity-preserving bounds with
 * alpha = 4). */
/* Interface flux schemes (Table tab:schemes_space), all on top of the GLM
 * interface values of (B_n, psi): HLL with Davis speed bounds; HLLD
 * (Miyoshi and Kusano 2005: contact, Alfven and fast waves, resolving
 * isolated contact and rotational discontinuities exactly); HLLC for MHD
 * (Li 2005: contact and fast waves, with the tangential field and velocity
 * of the star states from the HLL average; resolves isolated contacts). */
enum { AMRVAC_FLUX_HLL = 0, AMRVAC_FLUX_HLLD = 1, AMRVAC_FLUX_HLLC = 2 };

/* Grid and scheme description.  Physical boundary kinds per face follow the
 * paper's examples: periodic, zero-gradient ("continuous"), reflective
 * ((a)symmetric: normal momentum and normal field change sign) and a fixed
 * inflow state given in primitive variables. */
typedef struct {
  int ndim;               /* 2 or 3                                            */
  int block_nx;           /* interior cells per direction per block (even,     */
                          /* 4..16; the fused path and FP32-mixed need 16)     */
  int nghost;             /* ghost layers: 2, or 3 for the five-cell           */
                          /* reconstructions; block_nx >= 2 nghost            */
  int precision;          /* AMRVAC_FP64 or AMRVAC_FP32_MIXED                  */
  int base_blocks[3];     /* blocks per direction on level 1 (z ignored in 2D) */
  int bc_lo[3];           /* AMRVAC_BC_* at the minimum face of each direction */
  int bc_hi[3];           /* ... and at the maximum face (periodic must match) */
  int fix_small_values;   /* 0: flag small values only; 1: also replace them   */
  int reflux;             /* 1: coarse face flux := mean of fine face fluxes   */
  double xmin[3];         /* domain corner                                     */
  double xmax[3];
  double gamma;           /* adiabatic index                                   */
  double cfl;             /* Courant number C                                  */
  double glm_alpha;       /* psi damping: kappa = glm_alpha * c_h / min dx     */
  double small_density;   /* thresholds of the small-value check               */
  double small_pressure;
  double bc_fixed_prim[3][2][9]; /* primitive state of AMRVAC_BC_FIXED faces   */
  int limiter;            /* AMRVAC_LIM_*                                      */
  int flux;               /* AMRVAC_FLUX_*                                     */
} amrvac_grid_desc;

/* Device bytes of one state slot for nblocks blocks of this description.
 * Returns AMRVAC_E_ARG for an invalid description. */
int amrvac_slot_bytes(const amrvac_grid_desc* g, int nblocks, size_t* bytes);

/* Bytes before the first block in an FP64 slot (see the layout above). */
#define AMRVAC_SLOT_LEAD_FP64 16

/* Create a context on a block-based quadtree (2D) or octree (3D) hierarchy
 * with refinement ratio 2 (section "Open source strategy with MPI-AMRVAC");
 * only leaf blocks are advanced, with one time step for all levels.
 * level[nb] (1-based) and ijk[nb][3] (block position on
 * its level, z ignored in 2D) are HOST arrays describing the leaf blocks;
 * they must tile the domain without overlap and be 2:1 nested across faces,
 * edges and corners, else AMRVAC_E_ARG.  slots[nslots] are device pointers
 * of amrvac_slot_bytes each (nslots >= 3 for SSPRK(3,3) stepping); stream is
 * a hipStream_t (NULL = the null stream).  The library builds its neighbour
 * and ghost task tables on the host, uploads them and allocates its own
 * scratch (primitive and face-flux buffers, reduction scalars). */
int amrvac_init_blocks(amrvac_ctx** out, const amrvac_grid_desc* g, int nblocks,
                       const int* level, const int* ijk, void* const* slots, int nslots,
                       void* stream);

/* Convert a DEVICE array of primitive variables, [block][var][interior cell]
 * FP64 (block_nx^ndim cells per block, i fastest), to conserved variables in
 * the interior of slot.  Ghost cells are left untouched. */
int amrvac_set_primitive(amrvac_ctx* c, int slot, const double* prim_dev);

/* Copy the interior conserved state of slot into a DEVICE FP64 array
 * [block][var][interior cell]. */
int amrvac_get_conserved(amrvac_ctx* c, int slot, double* cons_dev);

/* Fill the face ghost slabs of slot that amrvac_stage reads on the selected
 * path: same-level copies with periodic wrap, restriction (pairwise-summed
 * volume average) of finer neighbours and physical boundaries, then limited
 * linear prolongation of coarser neighbours (the paper's internal boundary
 * exchange of the "Future directions" section, done on the device).  On
 * AMRVAC_PATH_PLAIN every face ghost slab is filled; on AMRVAC_PATH_FUSED
 * the stage and the prolongation read same-level neighbours in place, so
 * faces between same-level leaves are skipped. */
int amrvac_fill_ghosts(amrvac_ctx* c, int slot);

/* Time step from the interior of slot: dt = C / max_cells sum_d
 * (|v_d| + c_fast,d)/dx_d, then c_h = C / (dt * sum_d 1/dx_d) and kappa =
 * glm_alpha * c_h / min_d dx_d on the finest leaf level (CFL coupling of
 * the "Schemes and limiters" section).  Results go to DEVICE doubles; a
 * small value or an invalid dt sets the context's device flag word (read it
 * with amrvac_sync_flags).  No host synchronisation. */
int amrvac_cfl_dt(amrvac_ctx* c, int slot, double* dt_dev, double* ch_dev, double* kappa_dev);
/* (When the last call that wrote slot was amrvac_stage_cfl and its rate is
 * still held, only the final reduction runs; the result is identical.) */

/* One explicit stage (the advect1 statement of the IMEX implementation
 * section, with the SSPRK combination folded in):
 *   out = in + dt*L(in)                     if w == 1 (base not read),
 *   out = base + w*((in + dt*L(in)) - base) otherwise,
 * L = flux divergence of the van Leer + GLM + HLL interface fluxes plus the
 * psi damping source -kappa*psi.  dt, c_h, kappa are read from DEVICE
 * pointers (as written by amrvac_cfl_dt).  in must have had its ghosts
 * filled; in != out; out may equal base. */
int amrvac_stage(amrvac_ctx* c, int in_slot, int base_slot, int out_slot, double w,
                 const double* dt_dev, const double* ch_dev, const double* kappa_dev);

/* amrvac_stage that also folds the CFL rate of every output cell (the
 * quantity amrvac_cfl_dt maximises, from the values as stored) into the
 * context's per-job running maximum, so that a following amrvac_cfl_dt on
 * out_slot skips its pass over the state: the usual last stage of an SSPRK
 * step.  The held rate is dropped when anything else writes out_slot, when
 * amrvac_cfl_dt runs on another slot or when the block tables change.  On
 * grids with coarse/fine flux corrections (which change the coarse cells
 * next to finer leaves after the stage) those cells are folded in after the
 * correction.  On the plain path, and for 3D contexts with three ghost
 * layers (whose folding stage is no cheaper than the separate pass), it is
 * exactly amrvac_stage. */
int amrvac_stage_cfl(amrvac_ctx* c, int in_slot, int base_slot, int out_slot, double w,
                     const double* dt_dev, const double* ch_dev, const double* kappa_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * amrvac_stage on the per-kernel (plain) FP64 path, with the same arguments,
 * checks and result bit for bit, whose primitive and face-flux scratch is a
 * static device array of AMRVAC_NOALLOC_SCRATCH_BYTES held by each GPU from
 * the library's load until the process ends, instead of library allocations.
 * It calls no allocating routine.  It runs the per-kernel kernels whatever
 * path the context is set to; FP64 single-job contexts only (else
 * AMRVAC_E_ARG, batch contexts AMRVAC_E_STATE).  A grid whose scratch
 * (blocks x 9 x 8 B x (padded cells + ndim x faces per block), each part
 * rounded up to 256 B) exceeds the array is rejected with AMRVAC_E_ARG and
 * a message giving both sizes: 3D blocks of 16^3 need 1.52 MB each (up to
 * 44 blocks), 2D blocks of 16^2 68 KB (up to 987).  Every call on a GPU
 * shares that GPU's array: calls that overlap in time on one GPU (other
 * streams, other contexts, other threads) race and must be ordered by the
 * caller.  No part of the array needs to start cleared. */
#define AMRVAC_NOALLOC_SCRATCH_BYTES (64u << 20)
int amrvac_stage_noalloc(amrvac_ctx* c, int in_slot, int base_slot, int out_slot, double w,
                         const double* dt_dev, const double* ch_dev, const double* kappa_dev);

/* Two-state combination on the leaf interior cells of every block:
 *   out = a + coef*(b - a)
 * (arithmetic in double; FP32-mixed slots round the result to their storage
 * precision).  It is the stage-free row of a Shu-Osher scheme written around
 * a: the last SSPRK(5,4) stage takes its base state from it.  a, b and out
 * are slot indices; out may equal a or b (each cell reads its own values
 * before writing); ghost cells of out are not written.  AMRVAC_E_ARG for a
 * bad slot or a non-finite coef.  No host synchronisation. */
int amrvac_combine(amrvac_ctx* c, int a_slot, int b_slot, double coef, int out_slot);

/* Advance nsteps full SSP Runge-Kutta steps of slot 0 (Table
 * tab:schemes_time), using slots 1 .. 3 as stage storage and library-owned
 * dt/c_h/kappa; each step is cfl -> [fill -> stage] x nstages:
 *   nstages = 2: SSPRK(2,2), stage weights (1, 1/2);
 *   nstages = 3: SSPRK(3,3), stage weights (1, 1/4, 2/3);
 *   nstages = 4: SSPRK(4,3), four stages advancing by dt/2 each, weights
 *                (1, 1, 1/3, 1) (the third returns to the step's start);
 *   nstages = 5: SSPRK(5,4) of Spiteri and Ruuth, Shu-Osher coefficients:
 *                four stages around the step's start u0, then
 *                amrvac_combine(u0, u2) and a fifth stage from u4 with that
 *                base (its L(u3) term is carried by u4).  Needs 4 slots.
 * The last stage folds in the next step's CFL rate where it can
 * (amrvac_stage_cfl).  use_graph = 1 captures one step in a HIP graph on
 * first use and replays it.  No host synchronisation. */
int amrvac_advance(amrvac_ctx* c, int nsteps, int nstages, int use_graph);

/* ---------------------------------------------------------------------------
 * Regrid: change a single-job context's leaf set (the block-based AMR of the
 * "Open source strategy" section, with refinement ratio 2), each block
 * changing by at most one level.
 * -------------------------------------------------------------------------*/

/* Plan a new leaf set (host only; no context, no device work) from the
 * grid g and its current leaf set (nb blocks: level, ijk as in
 * amrvac_init_blocks): refine the blocks with flags[b] > 0 (levels capped
 * at max_level), restore 2:1 nesting over faces, edges and corners by
 * refining leaves that became two levels coarser than a neighbour, then
 * coarsen every complete set of 2^ndim sibling leaves that are all flagged
 * < 0, where the parent would not sit next to a leaf two levels finer.
 * Writes nb_new, and, when cap >= nb_new, the new blocks' levels and
 * positions (ijk_out: 3 ints per block) in (level, i, j, k) order;
 * AMRVAC_E_NOMEM (with nb_new set) when cap is too small, AMRVAC_E_ARG for
 * an invalid grid or leaf set (message in amrvac_last_error(NULL)). */
int amrvac_regrid_plan(const amrvac_grid_desc* g, int nb, const int* level, const int* ijk, const int* flags,
                       int max_level, int cap, int* nb_new, int* level_out, int* ijk_out);

/* Move the state in slot to a new leaf set and return a new context on
 * caller-owned slots for it (nslots slots of amrvac_slot_bytes(nb) bytes;
 * the state lands in its slot 0), with the old context's grid, path, launch
 * shape and stream.  Every new block must be an old block (copied), a child
 * of an old leaf (conservative linear prolongation: the parent value plus a
 * quarter of the minmod-limited parent slope per direction, as for the
 * ghost cells) or the parent of 2^ndim old leaves (their volume average,
 * pairwise sums); otherwise AMRVAC_E_ARG.  The old slot's ghost cells are
 * filled on the way; the old context is left usable and is not destroyed.
 * Synchronises the stream. */
int amrvac_regrid(amrvac_ctx* c, int slot, int nb, const int* level, const int* ijk, void* const* slots, int nslots,
                  amrvac_ctx** out);

/* Loehner's error indicator per leaf block, for refinement decisions (the
 * paper's runs refine on weighted, user-chosen plasma quantities; this is
 * the second-derivative estimator of Loehner 1987 in its per-direction form).
 * For every interior cell, conserved variable q and direction d, with a, b,
 * e the cell's lower neighbour, itself and its upper neighbour along d:
 *   E_q = sqrt( sum_d (a - 2b + e)^2 /
 *               sum_d (|e - b| + |b - a| + wavefilter (|e| + 2|b| + |a|))^2 )
 * (0 where the denominator is 0); indicator[b] = max over the block's cells
 * of sum_q weights[q] E_q.  Callers typically refine above a threshold
 * (0.1 - 0.2) and coarsen below a fraction of it.  A variable that is zero
 * up to roundoff gives a ratio of roundoff terms (order 1, not
 * reproducible): weight only variables that carry the solution.
 *   slot:          state to examine; its ghost cells are filled on the way
 *   weights:       host [9] in conserved order (rho, m, e, B, psi), finite,
 *                  >= 0, at least one positive
 *   wavefilter:    finite, >= 0 (0.01 is usual)
 *   indicator_dev: device [nb] doubles, caller-owned, block order of
 *                  amrvac_init_blocks; written asynchronously on the stream
 * AMRVAC_E_ARG for bad arguments, AMRVAC_E_STATE on batch contexts. */
int amrvac_lohner(amrvac_ctx* c, int slot, const double* weights, double wavefilter, double* indicator_dev);

/* Select the stage implementation: AMRVAC_PATH_PLAIN (separate primitive,
 * per-direction flux, reflux and update kernels; FP64 only, the default for
 * FP64 contexts) or AMRVAC_PATH_FUSED (one kernel per stage plus, on AMR
 * grids, a coarse/fine flux correction; needs block_nx = 16; the only path
 * of FP32-mixed contexts).
 * AMRVAC_E_ARG if the context cannot run it. */
int amrvac_set_path(amrvac_ctx* c, int path);

/* Launch shape of the fused stage.  Every shape gives bit-identical results;
 * they differ only in speed.
 *   zseg:   workgroups per 3D block, each marching 16/zseg of its z planes
 *           (1, 2 or 4; 1 in 2D).  More, shorter workgroups fill the GPU on
 *           small grids at the cost of re-reading 4 planes per segment.
 *   rotate: 1 rotates the per-plane extra work (halo cells, halo slopes and
 *           the 17th face of each line) over the four waves of a workgroup,
 *           0 leaves it to the first waves.
 *   xcd:    1 gives each of the 8 XCDs a contiguous run of the Morton-ordered
 *           block list (neighbours share an L2), 0 deals workgroups out in
 *           list order.
 * The default is {1, 0, 1}. */
typedef struct {
  int zseg;
  int rotate;
  int xcd;
} amrvac_tune;

#define AMRVAC_TUNE_MAX_CANDIDATES 12

/* Set / read the launch shape.  AMRVAC_E_ARG for an invalid shape.  A
 * change synchronises the stream and drops the captured step graph. */
int amrvac_set_tune(amrvac_ctx* c, const amrvac_tune* t);
int amrvac_get_tune(const amrvac_ctx* c, amrvac_tune* t);

/* Autotuner: time every launch shape (zseg-major, then rotate, then xcd;
 * 12 candidates in 3D, 4 in 2D) on this context's own grid, as reps fused
 * stages of weight 1 from in_slot into out_slot after one untimed launch,
 * with dt, c_h and kappa from the CFL of in_slot, and keep the fastest.
 * Needs a single-job context on the fused path.  out_slot is overwritten;
 * in_slot's ghost cells are filled; the flag word and fix count are left as
 * they were.  Synchronises the stream.  best (may be NULL) receives the
 * chosen shape, ms (may be NULL; AMRVAC_TUNE_MAX_CANDIDATES floats) the mean
 * time per launch of each candidate, ncand (may be NULL) their number. */
int amrvac_autotune(amrvac_ctx* c, int in_slot, int out_slot, int reps, amrvac_tune* best, float* ms, int* ncand);

/* Synchronise the stream and read the device flag word (AMRVAC_FLAG_* bits
 * accumulated since the last reset), the number of cells fixed by the
 * small-value fix, and the last dt written by amrvac_advance.  Returns
 * AMRVAC_E_NONPHYSICAL if a flag is set and fixes are off, else AMRVAC_OK.
 * Any pointer may be NULL. */
int amrvac_sync_flags(amrvac_ctx* c, int* flags_host, long long* nfix_host, double* dt_host);

/* Clear the device flag word and fix counter (enqueued on the stream). */
int amrvac_reset_flags(amrvac_ctx* c);

/* ---------------------------------------------------------------------------
 * Batch (serving) contexts: many independent jobs resident on the device,
 * advanced together.  A job is one grid of the same block shape, precision
 * and physics (gamma, small-value settings, fixed boundary states) as the
 * batch; it may differ in size, hierarchy, boundaries, Courant number and
 * step count.  Its blocks occupy a contiguous run of places in the batch's
 * block pool; each step advances every job with steps left by one
 * SSPRK(nstages) step with its own dt, c_h and kappa, in one launch per
 * kernel for all jobs (the fused path).  Jobs join and leave between steps.
 * -------------------------------------------------------------------------*/

/* Create a batch context.  shape supplies ndim, block_nx (must be 16),
 * nghost (2, or 3 for the five-cell reconstructions), precision
 * and the physics every job must share (including limiter and flux);
 * nstages as in
 * amrvac_advance; slots are 2 (nstages = 2), 3 (nstages = 3, 4) or 4 (nstages = 5)
 * caller-owned DEVICE buffers of
 * amrvac_slot_bytes(shape, capacity_blocks) bytes each (the block pool);
 * max_jobs bounds the number of resident jobs. */
int amrvac_batch_create(amrvac_ctx** out, const amrvac_grid_desc* shape, int capacity_blocks, int max_jobs,
                        int nstages, void* const* slots, void* stream);

/* Admit a job: validate its block table (as amrvac_init_blocks), place its
 * blocks in the first free run of the pool that fits, and convert its DEVICE
 * primitive state ([block][var][interior cell] FP64) into the pool.  It will
 * take nsteps steps.  *job_out receives the job id.  AMRVAC_E_NOMEM when no
 * job slot or no contiguous run of nblocks places is free (the caller keeps
 * it queued); AMRVAC_E_ARG when its shape or physics differs. */
int amrvac_batch_add_job(amrvac_ctx* c, const amrvac_grid_desc* g, int nblocks, const int* level, const int* ijk,
                         const double* prim_dev, int nsteps, int* job_out);

/* Enqueue one step of every job that has steps left.  No host sync, except
 * that admitting or finishing jobs makes the next step wait for the stream
 * while the block lists are rebuilt. */
int amrvac_batch_step(amrvac_ctx* c);

/* Host-side progress of a job (no device access). */
int amrvac_batch_job_info(amrvac_ctx* c, int job, int* steps_done, int* steps_left, int* nblocks);

/* Copy a job's interior conserved state to a DEVICE FP64 array
 * [block][var][interior cell] (enqueued on the stream). */
int amrvac_batch_get_job(amrvac_ctx* c, int job, double* cons_dev);

/* Retire a job and return its pool places (waits for the stream). */
int amrvac_batch_remove_job(amrvac_ctx* c, int job);

/* Largest free run and total free places of the pool. */
int amrvac_batch_free_blocks(amrvac_ctx* c, int* largest_run, int* total_free);

/* Message of the last failed call on this context (never NULL). */
const char* amrvac_last_error(const amrvac_ctx* c);

/* Synchronise, free library-owned memory and graphs.  Slots stay. */
int amrvac_destroy(amrvac_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* AMRVAC_H */
