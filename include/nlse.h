/*
 * nlse.h -- C ABI of libnlse, an MI355X (gfx950) integrator for the
 * nonlinear Schroedinger / Gross-Pitaevskii equation
 *
 *     i Psi_t + a Lap(Psi) - V Psi + s |Psi|^2 Psi = 0          (Eq. NLSE)
 *
 * advanced by classic RK4 (Eq. RK4) with the right-hand side
 * F(Psi) = i [ a L Psi + (s|Psi|^2 - V) Psi ], where L is the second-order
 * central difference (CD2, step 1 of Eqs. 2shoc1d / 2d2shocs1 / 3d2shocs) or
 * the fourth-order two-step compact scheme 2SHOC (Eqs. 2shoc1d2 / 2d2shocs2 /
 * 3d2shocs2), and boundary points follow Dirichlet (Eqs. BCDdt, BCDlap) or
 * modulus-squared Dirichlet (Eqs. msd, BCMSDlap) conditions.
 * (Caplan, "NLSEmagic", arXiv:1203.1263, Secs. "Finite-difference schemes",
 * "Boundary conditions", "Stability".)
 *
 * Conventions for every function below
 * -------------------------------------
 *  - Grids: ndim in {1,2,3}; dims = {Nx, Ny, Nz}, entries beyond ndim must be
 *    1; every active extent must be >= 3.  Equal spacing h in all directions
 *    (Sec. "Finite-difference schemes").  Every point with an active index 0
 *    or N-1 is a boundary point.
 *  - Layout: interleaved complex (re, im), x fastest, linear index
 *    x + Nx*(y + Ny*z); FP32 fields are float2 arrays, FP64 fields double2.
 *    A potential V is a real array of the same element type and shape.
 *  - Device pointers are HIP device addresses (e.g. from a torch CUDA tensor
 *    under ROCm); "borrowed" buffers stay owned by the caller and must
 *    outlive the object that references them.
 *  - Streams: hip_stream is a hipStream_t passed as void*; NULL = the legacy
 *    default stream.  All work is enqueued asynchronously on that stream
 *    unless a function says it synchronises.
 *  - Errors: 0 on success, a negative nlse_status otherwise.  Arguments are
 *    validated before anything is launched; on error nothing was enqueued.
 *    nlse_last_error() returns a thread-local message for the last failure.
 *  - Threading: objects are not internally locked; use one object per host
 *    thread (or serialise calls).  Different objects are independent.
 */
#ifndef NLSE_H_
#define NLSE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ constants */

typedef enum {
    NLSE_OK = 0,
    NLSE_EINVAL = -1,      /* bad argument (shape, parameter, pointer, size)  */
    NLSE_ENOMEM = -2,      /* host allocation failed / workspace too small    */
    NLSE_EDEVICE = -3,     /* a HIP runtime call failed (message has details) */
    NLSE_EUNSTABLE = -4,   /* non-finite mass or energy: the run blew up      */
    NLSE_EUNSUPPORTED = -5 /* valid but not implemented combination          */
} nlse_status;

enum { NLSE_F32 = 0, NLSE_F64 = 1 };               /* element type            */
enum { NLSE_CD2 = 2, NLSE_2SHOC = 4 };              /* Laplacian order         */
/* Boundary conditions (Sec. "Boundary conditions"), each applied through its
 * time form to F at boundary points and, for 2SHOC, through its Laplacian
 * form to the step-1 value D at boundary points:
 *   NLSE_BC_DIRICHLET  Eqs. BCDdt / BCDlap: F_b = 0, D_b = -(1/a) N_b Psi_b
 *   NLSE_BC_MSD        Eqs. msd / BCMSDlap: F_b from the inward neighbour q,
 *                      F_b = i Im(F_q/Psi_q) Psi_b (q one step inward on
 *                      every boundary axis; a zero Psi_q gives 0)
 *   NLSE_BC_L0         Eqs. BCL0dt / BCL0lap: F_b = i N_b Psi_b, D_b = 0
 * with N = s|Psi|^2 - V.  Boundary points: an index 0 or N_d-1 on any axis. */
enum { NLSE_BC_DIRICHLET = 0, NLSE_BC_MSD = 1, NLSE_BC_L0 = 2 };

/* Grid / batch flags. */
#define NLSE_COMPENSATED 0x1u /* FP32 only: keep Psi as hi+lo pair, RK4
                                 combination of the last stage done in FP64 */
#define NLSE_NO_GRAPH 0x2u    /* grid or batch: launch directly instead of
                                 replaying captured HIP graphs */
#define NLSE_FUSED_PAIRS 0x4u /* grid only: run each pair of RK4 steps as
                                 four stage-pair launches (stages 1+2, 3+4
                                 per step) that keep U1 and U3 on chip (80
                                 instead of 168 B per point-step compensated,
                                 same bits); an odd last step takes four
                                 passes.  2D grids: every type, scheme and
                                 boundary condition, on the 64x16 tile if it
                                 is the grid's, else 32x32.  3D grids: FP32
                                 2SHOC, Dirichlet / MSD, on the 32x8 tile
                                 (slower than four passes there: 2
                                 workgroups per CU).  Off by default. */

typedef struct nlse_grid nlse_grid;

/* ------------------------------------------------------------ utilities */

/* Linear stability bound of RK4 with CD2 (Eq. stblincd):
 *     k < h^2 / (ndim sqrt(2) a),
 * and 3/4 of it for 2SHOC (Eq. stblin2shoc).  No safety factor is applied
 * (the paper's drivers multiply by 0.8).  Returns a negative value for
 * invalid arguments. */
double nlse_dt_max(int ndim, int order, double h, double a);

/* Human-readable text for a status code (static storage). */
const char *nlse_strerror(int status);

/* Thread-local detail message of the last failing call on this thread. */
const char *nlse_last_error(void);

/* ------------------------------------------------------------ single grid */

/* Size in bytes of the device workspace a grid needs: the RK4 accumulator,
 * two ping-pong stage buffers, the FP32 compensation term (if
 * NLSE_COMPENSATED) and reduction partials.  dims as described above. */
int nlse_workspace_bytes(int ndim, const int64_t dims[3], int dtype,
                         unsigned flags, size_t *bytes);

/* Create a grid.
 *   psi_dev   device buffer of Npts complex values (borrowed; updated in place
 *             by nlse_step_rk4).
 *   work_dev  device buffer of >= nlse_workspace_bytes() bytes, 256-byte
 *             aligned (borrowed; its contents are owned by the grid).
 *   h, a, s   spacing, dispersion a > 0, nonlinearity s (finite).
 *   flags     0, NLSE_COMPENSATED (FP32 only), NLSE_FUSED_PAIRS,
 *             NLSE_NO_GRAPH.
 * The compensation term starts at zero.  Enqueues its initialisation on the
 * stream.  On success *g receives the new grid. */
int nlse_create_grid(nlse_grid **g, int ndim, const int64_t dims[3], double h,
                     double a, double s, int dtype, unsigned flags,
                     void *psi_dev, void *work_dev, size_t work_bytes,
                     void *hip_stream);

/* Set (V_dev != NULL, borrowed, real, same element type and shape) or clear
 * (V_dev == NULL, meaning V == 0) the external potential of Eq. NLSE. */
int nlse_set_potential(nlse_grid *g, const void *V_dev);

/* Advance nsteps classic RK4 steps of size dt (Eq. RK4) with Laplacian
 * `order` (NLSE_CD2 or NLSE_2SHOC) and boundary condition `bc`.  Each step is
 * four fused stage kernels (stencil, boundary update and RK4 accumulation in
 * one pass each); grids created with NLSE_FUSED_PAIRS run two launches per
 * step instead (stages 1+2 and 3+4), with the same bits (NLSE_BC_L0 always
 * takes the four single-stage kernels).  Unless the grid
 * has NLSE_NO_GRAPH, the launches of up to 64 steps are captured once per
 * (order, bc, dt, tile, step count) into a HIP graph that is replayed
 * (setting a different potential drops the captured graphs).
 * Psi is updated in place; asynchronous.  dt > 0 finite,
 * nsteps >= 0.  A dt above nlse_dt_max() is allowed (blow-up shows up as
 * NLSE_EUNSTABLE from nlse_mass_energy). */
int nlse_step_rk4(nlse_grid *g, int order, int bc, double dt, int64_t nsteps);

/* Frames (Sec. "Chunk-size Limitations": the integrator hands the field back
 * to the host every `chunk` steps).  Runs nframes chunks of `chunk` RK4 steps
 * (as nlse_step_rk4) and copies the field after chunk j into
 * frames_host + j * npts elements (interleaved complex of the grid's element
 * type; for NLSE_COMPENSATED grids the stored FP32 field).  The copies
 * overlap the integration: after each chunk Psi is copied device to device,
 * on the grid's stream, into one half of stage_dev (caller-owned device
 * memory, 16-byte aligned, stage_bytes >= 2 * npts * element bytes), and a
 * library-owned stream moves that half to the host while the next chunk
 * runs (the calling thread orders the two streams, waiting on events).  frames_host (caller-owned, nframes * npts elements) should be
 * pinned (hipHostMalloc) for the overlap; pageable memory gives the same
 * frames, copied without overlap.  Synchronises: returns after the last
 * frame is on the host.  chunk >= 1, nframes >= 0 (0: no work). */
int nlse_run_frames(nlse_grid *g, int order, int bc, double dt, int64_t chunk,
                    int64_t nframes, void *frames_host, void *stage_dev,
                    size_t stage_bytes);

/* Mass M = h^d sum |Psi|^2 and energy
 *   E = h^d [ sum_interior -a Re(conj(Psi) L Psi) + sum ( V|Psi|^2 - (s/2)|Psi|^4 ) ]
 * (the standard NLSE invariants; the paper defines neither), with L the
 * scheme Laplacian of `order` (2SHOC uses the boundary D of `bc`).  Partial
 * sums in FP64 per workgroup over a fixed partition, then a fixed-order final
 * sum: the result is bitwise reproducible.  Synchronises the stream.
 * Returns NLSE_EUNSTABLE (after writing both values) if either is not
 * finite. */
int nlse_mass_energy(nlse_grid *g, int order, int bc, double *mass,
                     double *energy);

/* Mass and energy of a field without a grid and without any device
 * allocation: for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Computes exactly what nlse_mass_energy computes for a grid of this shape,
 * these parameters and this potential (the same bits): psi_dev holds Npts
 * interleaved complex values of dtype, V_dev a real array of the same shape
 * or NULL (V == 0); both are only read.  Where nlse_mass_energy stores the
 * 2SHOC step-1 values D in the grid's workspace, this one recomputes D at
 * each point where the Laplacian needs it (about 3x slower in 3D).  Scratch:
 * the per-workgroup partial sums and the three result doubles live in a
 * library-owned static device array of 1.5 MiB (one per device, kept until
 * the process ends), which limits fields to 2^28 points (larger:
 * NLSE_EINVAL, nothing launched).  Every value in it is written before it is
 * read in the same call, so nothing needs clearing.  Calls that overlap on
 * one device (several host threads, or streams running concurrently) share
 * that array and race: serialise them.  No hipMalloc, hipFree or other
 * allocating call is made.  Runs on hip_stream (NULL = default stream) and
 * synchronises it; returns NLSE_EUNSTABLE (after writing both values) if
 * either is not finite. */
int nlse_mass_energy_noalloc(int ndim, const int64_t dims[3], double h,
                             double a, double s, int dtype, int order, int bc,
                             const void *psi_dev, const void *V_dev,
                             void *hip_stream, double *mass, double *energy);

/* Copy the compensation term (Npts complex FP32 values, same layout as Psi)
 * out to / in from a device buffer.  lo_dev == NULL in nlse_set_state resets
 * it to zero (call this after overwriting Psi).  Grids without
 * NLSE_COMPENSATED return NLSE_EINVAL.  Asynchronous. */
int nlse_get_state(nlse_grid *g, void *lo_dev);
int nlse_set_state(nlse_grid *g, const void *lo_dev);

/* Tile shape used by the stage kernels: (tx, ty, cz) = x-width, y-height and
 * z-chunk length (unused entries 1).  Any supported shape gives bitwise
 * identical results.  1D: 256 runs each stage as a kernel; 1024 (the
 * default for grids of at most 1024 FP64 / 2048 FP32 points) runs every
 * step of a call in one on-chip workgroup.  nlse_autotune times the candidates for
 * (order, bc) on this grid (running stage kernels on scratch copies, the
 * field is not changed; for fused 3D grids only the z-chunk of the 32x8
 * tile is tuned, for 2D grids with NLSE_FUSED_PAIRS the pair tile, 32x32
 * or 64x16), keeps the fastest and stores it in the cache file
 * named by $NLSE_TUNE_CACHE if set.  On 2D grids without NLSE_FUSED_PAIRS
 * it also times the first stage pair on both pair tiles against stages 1
 * and 2 on the best four-pass tile, and runs later steps of this order as
 * stage pairs if they were faster (the same bits; see NLSE_FUSED_PAIRS).
 * nlse_set_tile forces a shape run as four passes unless the grid has
 * NLSE_FUSED_PAIRS (NLSE_EUNSUPPORTED if it is not a compiled candidate).
 * nlse_get_stage_pairs sets *on to 1 if steps of `order` run as stage pairs
 * with the current settings (3D: except under the L0 condition). */
int nlse_autotune(nlse_grid *g, int order, int bc, double dt);
int nlse_get_tile(const nlse_grid *g, int order, int tile[3]);
int nlse_set_tile(nlse_grid *g, int order, const int tile[3]);
int nlse_get_stage_pairs(const nlse_grid *g, int order, int *on);

/* Destroy a grid: frees library-internal host objects and graphs only. */
int nlse_destroy_grid(nlse_grid *g);

/* ------------------------------------------------------------ batches */

/* Many independent 2D problems of uneven size and parameters advanced
 * together by one persistent launch per nlse_batch_step_rk4 call (captured
 * once into a HIP graph per step count and replayed).  Every problem follows
 * exactly the single-grid integrator above (same scheme, boundary forms and
 * RK4 stages, Eq. RK4 / Eq. RK4_GPU) with its own a, s, V, h, dt, order and
 * bc; a problem gives bitwise the same result alone (with the batch's
 * tile) as inside a batch.  Only 2D problems are supported (NLSE_EUNSUPPORTED otherwise). */
typedef struct {
    int ndim;            /* must be 2                                       */
    int64_t dims[3];     /* {Nx, Ny, 1}, Nx, Ny >= 3                        */
    double h, a, s, dt;  /* spacing, dispersion (> 0), nonlinearity, step   */
    int order, bc;       /* NLSE_CD2 / NLSE_2SHOC, NLSE_BC_DIRICHLET / _MSD / _L0 */
    int64_t psi_offset;  /* first complex element of this field in psi_pool */
    int64_t v_offset;    /* first real element of V in v_pool, -1: V == 0   */
} nlse_sim_desc;

typedef struct nlse_batch nlse_batch;

/* Workspace bytes for a batch (accumulator, stage buffers, compensation,
 * schedule, reduction scratch). */
int nlse_batch_workspace_bytes(int nsims, const nlse_sim_desc *sims, int dtype,
                               unsigned flags, size_t *bytes);

/* Create a batch.  psi_pool (psi_pool_elems complex values) and v_pool
 * (v_pool_elems reals, may be NULL if every v_offset is -1) are borrowed
 * device pools; each problem's field must lie inside psi_pool and fields must
 * not overlap (not checked).  work_dev: >= nlse_batch_workspace_bytes bytes,
 * 256-byte aligned, borrowed.  flags: NLSE_COMPENSATED (FP32), NLSE_NO_GRAPH.
 * Builds a cost-balanced static schedule of (problem, tile) items over the
 * persistent workgroups (tile 32x8, 3 per CU until reconfigured, see
 * nlse_batch_set_config); synchronises the stream. */
int nlse_batch_create(nlse_batch **b, int nsims, const nlse_sim_desc *sims,
                      int dtype, unsigned flags, void *psi_pool,
                      size_t psi_pool_elems, const void *v_pool,
                      size_t v_pool_elems, void *work_dev, size_t work_bytes,
                      void *hip_stream);

/* Advance every problem nsteps RK4 steps with its own dt (asynchronous, one
 * persistent launch), 0 <= nsteps <= 2^24 (NLSE_EINVAL otherwise, checked
 * first).  Workgroups that share a problem meet at a barrier after every
 * pass (a stage, or a stage pair), counted in 64-bit arrival counters (the
 * last target of a call, at most 4 nsteps x group size, cannot wrap); a wait
 * there is bounded (about 2^25 polls, or the value of $NLSE_BATCH_SPIN_LIMIT
 * read at creation), and one that runs out sets an error flag read by
 * nlse_batch_status, after which every waiting workgroup leaves the kernel.
 * With stage pairs (nlse_batch_set_config) Psi alternates between psi_pool
 * and the workspace inside a call and is back in psi_pool when it returns. */
int nlse_batch_step_rk4(nlse_batch *b, int64_t nsteps);

/* Per-problem mass and energy (as nlse_mass_energy, with each problem's own
 * order and bc) into host arrays of nsims doubles.  Synchronises. */
int nlse_batch_mass_energy(nlse_batch *b, double *mass, double *energy);

/* Synchronises; NLSE_EDEVICE if a barrier of the persistent kernel timed
 * out since creation (the fields are then not valid), else NLSE_OK. */
int nlse_batch_status(nlse_batch *b);

/* Tile (tx x ty: 32x8, 64x4, 64x8, 128x4, 64x16, 32x16 or 32x32), persistent workgroups
 * per CU (1..16; the grid holds min(wg_per_cu, what fits on a CU) x CUs
 * workgroups) and pass structure of the batched kernel: pairs = 0 runs the
 * four RK4 stages as four passes over the batch, pairs = 1 as two passes of
 * two stages (1+2, 3+4; each tile evaluates the first stage of a pair on
 * itself and the halo ring the second stage reads, so the intermediate
 * stage never goes through memory; with an odd nsteps the first step of a
 * call takes three passes).  Any configuration gives bitwise the same
 * fields as single grids with that tile.  nlse_batch_set_config rebuilds
 * the static schedule for it (synchronises; NLSE_EUNSUPPORTED for a tile
 * that is not compiled, NLSE_EINVAL for pairs other than 0 or 1).  Created
 * batches use 32x8, 3 per CU, pairs = 0.  nlse_batch_autotune times whole
 * RK4 steps of every tile with 1..5 workgroups per CU (up to what fits) and
 * pairs 0 and 1 on this batch; it saves Psi and the compensation term to a
 * temporary device allocation of (1 or 2) x total points x element size
 * first and restores them afterwards, so the fields are not changed.  It
 * keeps the fastest and stores it in the cache file named by
 * $NLSE_TUNE_CACHE if set (a cached choice for the same problem shapes,
 * schemes and boundary conditions is reused without timing).
 * cfg = {tx, ty, wg_per_cu, pairs}. */
int nlse_batch_set_config(nlse_batch *b, int tx, int ty, int wg_per_cu, int pairs);
int nlse_batch_get_config(const nlse_batch *b, int cfg[4]);
int nlse_batch_autotune(nlse_batch *b);

/* info[0..3] = workgroups of the persistent launch, work items, total grid
 * points, captured graphs. */
int nlse_batch_info(const nlse_batch *b, int64_t info[4]);

int nlse_batch_destroy(nlse_batch *b);

/* ------------------------------------------------------------ surrogate */

/* A learned surrogate of kSteps = 16 RK4 steps of 2D fields (FP32 complex,
 * H x W, both multiples of 16): a 6-layer 3x3 convolutional residual network
 * on the two real channels, 2 -> 48 -> 48 -> 48 -> 48 -> 48 -> 2, ReLU after
 * layers 1-5, zero "same" padding, pred = psi + net(psi).  BF16 weights and
 * activations, FP32 accumulation on the matrix cores, FP32 master weights.
 * Not part of the paper's method: it is trained on trajectories of the
 * integrator above, which stays its fallback and the reference its error is
 * measured against.
 *
 * Parameters: one FP32 device array of nlse_surrogate_param_count() values,
 * per layer W (Cout, Cin, 3, 3) row-major then b (Cout), layers in order.
 * It is borrowed; nlse_surrogate_train_step updates it in place. */
typedef struct nlse_surrogate nlse_surrogate;

int nlse_surrogate_param_count(void);

/* Workspace for fields of H x W and batches up to max_batch (activations of
 * every layer, gradients, Adam moments, reduction scratch). */
int nlse_surrogate_workspace_bytes(int H, int W, int max_batch, size_t *bytes);

/* h: grid spacing (for masses).  Converts the weights to the kernel layouts
 * and zeroes the Adam moments (asynchronous on hip_stream). */
int nlse_surrogate_create(nlse_surrogate **m, int H, int W, int max_batch,
                          double h, float *params_dev, void *work_dev,
                          size_t work_bytes, void *hip_stream);

/* Call after the caller rewrote params_dev: rebuilds the BF16 weights and
 * resets the optimiser. */
int nlse_surrogate_refresh(nlse_surrogate *m);

/* psi_out = psi_in + net(psi_in) for `batch` contiguous complex64 fields
 * [batch][H][W]; psi_out must not alias psi_in. */
int nlse_surrogate_forward(nlse_surrogate *m, const void *psi_in,
                           void *psi_out, int batch);

/* Loss = mean over fields, points and the 2 real channels of
 * (pred - target)^2 and its gradient w.r.t. every parameter, written to
 * grad_dev (FP32, parameter layout) or, if NULL, kept internally.  The weight
 * gradient is summed in a fixed order (bitwise reproducible).  If loss is not
 * NULL the call synchronises and returns the loss. */
int nlse_surrogate_loss_grad(nlse_surrogate *m, const void *psi_in,
                             const void *psi_target, int batch,
                             float *grad_dev, double *loss);

/* One Adam step (b1 = 0.9, b2 = 0.999, eps = 1e-8) on the loss above with
 * learning rate lr; loss (pre-update) returned if not NULL (synchronises). */
int nlse_surrogate_train_step(nlse_surrogate *m, const void *psi_in,
                              const void *psi_target, int batch, float lr,
                              double *loss);

/* Masses h^2 sum |psi|^2 of `batch` fields into a host array (FP64, fixed
 * order; synchronises). */
int nlse_surrogate_field_mass(nlse_surrogate *m, const void *psi, int batch,
                              double *mass);

/* Boundary points of psi_out keep their phase and take the modulus of
 * psi_in (the fixed modulus of the MSD condition, Eq. BCMSDdef). */
int nlse_surrogate_project_msd(nlse_surrogate *m, const void *psi_in,
                               void *psi_out, int batch);

/* One surrogate block on `batch` fields in one pass: psi_out = psi_in +
 * net(psi_in), with (project_msd != 0) the boundary ring projected as
 * nlse_surrogate_project_msd does (same bits), and the masses
 * h^2 sum |psi_out|^2 of the results into the host array mass (batch
 * doubles).  The last layer does the projection and per-tile FP64 sums of
 * |psi_out|^2 in its epilogue, and a fixed-order pass adds the tiles of each
 * field (bitwise reproducible; the summation order differs from
 * nlse_surrogate_field_mass, so the last bits may).  psi_out must not alias
 * psi_in.  Synchronises. */
int nlse_surrogate_block(nlse_surrogate *m, const void *psi_in, void *psi_out,
                         int batch, int project_msd, double *mass);

/* Advance a 2D FP32 grid (same H x W, same stream) by nblocks blocks of 16
 * RK4 steps of size dt: each block is one surrogate evaluation (plus the MSD
 * projection when bc is NLSE_BC_MSD); if the relative mass drift of the block
 * exceeds drift_tol the block is discarded and recomputed by nlse_step_rk4
 * (order, bc, dt, 16).  Each block is one nlse_surrogate_block pass.  *n_fallbacks receives the number of such blocks.
 * Synchronises once or twice per block. */
int nlse_surrogate_advance(nlse_surrogate *m, nlse_grid *g, int order, int bc,
                           double dt, int64_t nblocks, double drift_tol,
                           int64_t *n_fallbacks);

/* Which kernels evaluate the network in nlse_surrogate_forward,
 * nlse_surrogate_block and nlse_surrogate_advance (training always uses the
 * layer-by-layer kernels, whose activations the backward pass reads):
 *   NLSE_SG_PATH_AUTO   whole-network pass for batches of at most
 *                       nlse_surrogate_fused_max_batch fields, else layers;
 *   NLSE_SG_PATH_LAYERS one kernel per layer, activations through HBM;
 *   NLSE_SG_PATH_FUSED  one kernel for all six layers: each workgroup takes a
 *                       16 x 16 output tile through every layer with the
 *                       activations in LDS, recomputing a ring of up to 5
 *                       pixels per layer (1.8x the flops, no activation
 *                       traffic, one launch).
 * Both paths give the same bits (the same operands, MFMAs and epilogue
 * operations in the same order).  Default: AUTO. */
#define NLSE_SG_PATH_AUTO 0
#define NLSE_SG_PATH_LAYERS 1
#define NLSE_SG_PATH_FUSED 2
int nlse_surrogate_set_path(nlse_surrogate *m, int path);
/* Largest batch that NLSE_SG_PATH_AUTO sends through the whole-network
 * kernel for this model's H x W. */
int nlse_surrogate_fused_max_batch(const nlse_surrogate *m);

int nlse_surrogate_destroy(nlse_surrogate *m);

#ifdef __cplusplus
}
#endif

#endif /* NLSE_H_ */
