/*
 * gsis.h -- C-ABI of libgsis.so, the MI355X (gfx950) kinetic hot path of the
 * general synthetic iterative scheme (GSIS) of arXiv 2310.18916, "Efficient
 * parallel solver for rarefied gas flow using GSIS".
 *
 * One kinetic pass (gsis_kinetic_step) builds, for every fluid cell and
 * velocity node, the Shakhov (monatomic) or Rykov two-VDF (diatomic)
 * reference distribution of Sec. 2.2, solves the implicit first-order upwind
 * transport system of Sec. 3.2 (Eq. delta_equations with first-order fluxes
 * on both sides) exactly by upwind sweeps, and reduces the distribution to
 * the moments of Eq. (getmoment).  gsis_gsis_correct runs the GSIS-II
 * macroscopic synthetic solve of Sec. 3.3 and schedules the VDF update of
 * Eq. (updatef); gsis_residual evaluates the convergence criterion of Sec. 5,
 * Eq. (convergence_critertion).
 * The calls mirror the Require/Ensure lists of Algorithms 1-3: the kinetic
 * solver takes f and returns W, the high-order terms and the boundary flux;
 * the macroscopic solver takes those and returns W.
 *
 * Units are dimensionless: lengths in L, molecular velocity in the most
 * probable speed sqrt(2 R T0), density in rho0, temperature in T0.
 *
 * Conventions for every call:
 *  - Every call returns gsis_status; nothing throws or aborts across the ABI.
 *    On an error the message is available from gsis_last_error(ctx).
 *  - All argument checks run on the host before any device work.
 *  - The library owns host metadata only.  Device memory is caller owned:
 *    query gsis_workspace_size, allocate that many bytes on the GPU (256-byte
 *    aligned) and pass them to gsis_bind_workspace.  The library never calls
 *    hipMalloc.
 *  - Device work is asynchronous on the bound stream (gsis_set_stream) except
 *    where a call says it synchronises.
 *  - One context per host thread; calls on one context must not overlap.
 *  - Canonical external layouts: cells x fastest, c = i + nx (j + ny k);
 *    velocity nodes x fastest, v = kx + nvx (ky + nvy kz) (a node list: its
 *    own order); a VDF is [cell][node].  The internal octant-grouped VDF
 *    layout is not exposed.
 */
#ifndef GSIS_H
#define GSIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsis_ctx gsis_ctx;

typedef enum {
    GSIS_OK = 0,
    GSIS_EINVAL = -1,      /* bad argument or configuration */
    GSIS_ESTATE = -2,      /* call out of order (e.g. step before init) */
    GSIS_ENOMEM = -3,      /* workspace too small, or host allocation failed */
    GSIS_EDEVICE = -4,     /* HIP runtime error */
    GSIS_ENOTFINITE = -5,  /* a non-positive or non-finite density/temperature appeared */
    GSIS_EDIVERGED = -6    /* residual grew beyond the divergence factor */
} gsis_status;

enum { GSIS_MONATOMIC = 0, GSIS_DIATOMIC = 1 };
enum { GSIS_FP64 = 0, GSIS_FP32 = 1 };
enum { GSIS_DIFFUSE_WALL = 0, GSIS_MAXWELL_INFLOW = 1 };
/* macroscopic boundary flux of gsis_gsis_correct (gsis_set_wall_flux) */
enum { GSIS_WALLFLUX_MAXWELL = 0, GSIS_WALLFLUX_G13 = 1 };
/* boundary slots for gsis_set_boundary: box faces, then the solid surface */
enum { GSIS_FACE_XM = 0, GSIS_FACE_XP = 1, GSIS_FACE_YM = 2, GSIS_FACE_YP = 3,
       GSIS_FACE_ZM = 4, GSIS_FACE_ZP = 5, GSIS_FACE_SOLID = 6 };

/* Number of FP64 values per cell returned by gsis_moments:
 * rho, ux, uy, uz, Tt, sxx, syy, szz, sxy, sxz, syz, qx, qy, qz
 * and, diatomic only, Tr, qrx, qry, qrz (Eq. getmoment; sigma in p0, q in p0 v_m). */
#define GSIS_NMOM_MONATOMIC 14
#define GSIS_NMOM_DIATOMIC 18

typedef struct {
    int nx, ny, nz;            /* uniform hex cells; h = l / n per axis */
    double lx, ly, lz;
    int nvx, nvy, nvz;         /* tensor velocity grid, >= 2 nodes per axis */
    double vmin[3], vmax[3];   /* node k at vmin + k (vmax - vmin)/(n - 1), trapezoid weights */
    int species;               /* GSIS_MONATOMIC (Shakhov, Pr = 2/3) or GSIS_DIATOMIC (Rykov) */
    double Kn;                 /* Knudsen number of Sec. 2.1; delta = sqrt(pi) / (2 Kn) */
    double omega;              /* viscosity index, mu ~ Tt^omega */
    double dr, Zr, A[4];       /* diatomic: internal DOF, rotational collision number,
                                  heat-flux relaxation rates A_tt, A_tr, A_rt, A_rr */
    double inv_dt;             /* 1/Delta t of the kinetic update; 0 = source iteration */
    int vdf_dtype;             /* GSIS_FP64 or GSIS_FP32 storage and sweep arithmetic */
    int conservative;          /* 1: reference distribution corrected to conserve the
                                  discrete mass, momentum and energy exactly */
    double macro_cfl;          /* pseudo-time CFL of the macroscopic iteration (e.g. 10) */
    int order;                 /* interface values of the explicit flux divergence of the
                                  kinetic update (Sec. 3.2): 0 or 1 first-order upwind; 2
                                  reconstructed to second order from the upwind cell with a
                                  least-squares gradient and the Venkatakrishnan limiter
                                  (faces on the box or a solid stay first order); the
                                  implicit increments stay first-order upwind either way.
                                  Order 2 adds two VDF-sized buffers (four diatomic) to the
                                  workspace and is not accepted by gsis_batch_create */
    double limiter_k;          /* order 2: Venkatakrishnan constant K, eps^2 = (K h)^3 S^2 with
                                  h the cube root of the cell volume and S the largest |f| of
                                  the point's stencil (the cell and its fluid neighbours);
                                  K < 0: no limiter */
} gsis_config;

/* Create a context for cfg.  Validates sizes (n >= 1, nv >= 2, vmax > vmin,
 * Kn > 0, lengths > 0; diatomic: dr > 0, Zr >= 1, A invertible).  All
 * boundaries default to a diffuse wall at rest with T = 1.  *out is NULL on
 * error. */
gsis_status gsis_create(gsis_ctx **out, const gsis_config *cfg);

/* Free the context (host memory only; the caller frees the workspace). */
gsis_status gsis_destroy(gsis_ctx *ctx);

/* Host array of n = nx*ny*nz bytes, 1 = solid cell, 0 = fluid.  Must precede
 * gsis_workspace_size.  Solid cells carry no VDF update and report NaN. */
gsis_status gsis_set_solid_mask(gsis_ctx *ctx, const uint8_t *mask, size_t n);

/* Non-uniform Cartesian velocity grid (Sec. 3.1 allows non-uniform Cartesian
 * grids; a tensor-product step towards its locally refined velocity meshes):
 * axis (0, 1, 2) gets the n host nodes given (n = the
 * configured nvx, nvy or nvz; finite, strictly increasing; copied) instead of
 * the uniform nodes on [vmin, vmax], with trapezoid weights (half of each
 * neighbouring gap).  The grid stays a tensor product, so every separable sum
 * keeps working.  Must precede gsis_workspace_size; EINVAL on a bad axis,
 * count or node array, ESTATE once the workspace is sized. */
gsis_status gsis_set_velocity_nodes(gsis_ctx *ctx, int axis, const double *nodes, int n);

/* General velocity set (Sec. 3.1: a locally refined or unstructured velocity
 * mesh, whose cells are represented by one node each): nodes is a host array
 * [n][4] of (xi_x, xi_y, xi_z, w), w > 0 the volume of the node's velocity
 * cell (the quadrature weight); copied.  Replaces the tensor grid of the
 * configuration: the node count becomes n (2 <= n <= 2^24) and canonical
 * node k is entry k of the list (gsis_get_vdf, gsis_set_vdf,
 * gsis_get_vdf_nodes).  Nothing factors per axis any more, so moments,
 * relaxation parameters and equilibrium wall fluxes are summed node by node.
 * Not accepted by gsis_batch_create.  Must precede gsis_workspace_size;
 * EINVAL on a bad count or a non-finite node or weight, ESTATE once the
 * workspace is sized (and from gsis_set_velocity_nodes afterwards). */
gsis_status gsis_set_velocity_list(gsis_ctx *ctx, const double *nodes, int n);

/* Unstructured spatial mesh (Sec. 3.2: the kinetic update of Eq.
 * (delta_equations) on cells i of volume V_i whose interfaces ij have area
 * S_ij and unit normal n_ij pointing from i to j; the paper's hypersonic
 * cases use tetrahedral and mixed-element meshes).  Host arrays, copied:
 * volume[ncell] > 0; face_cell[nface][2] = (owner cell, neighbour cell or
 * -1 - slot for a boundary face of boundary slot 0..6, whose condition
 * gsis_set_boundary gives); face_geom[nface][4] = (area >= 0, unit normal
 * out of the owner); cell_center[ncell][3] and face_center[nface][3] the
 * centroids (both NULL: kinetic passes only, no macroscopic correction).
 * Replaces the box of hex cells of the configuration (its nx, ny, nz, lx,
 * ly, lz are then unused; cells are numbered as given, gsis_moments has
 * ncell rows) and runs the first-order update, solved exactly: the library
 * groups the velocity nodes into classes that agree on the sign of xi . n
 * for every face orientation of the mesh and sorts each class's upwind graph
 * into levels, swept one after another.  gsis_gsis_correct solves the GSIS-II
 * equations of Sec. 3.3 on the same cells (least-squares velocity gradients
 * over the face neighbours, face gradients corrected along the line of the
 * two centroids, fluxes per unit area times S/V, the high-order terms of each
 * face from the kinetic face flux).  Requires gsis_set_velocity_list first,
 * order 1 and no solid mask (a body is a hole in the mesh, its surface
 * boundary slot 6); must precede gsis_workspace_size.  Kinetic passes,
 * moments, residual (volume-weighted), gsis_precondition (the Euler form of
 * the same solve) and state calls work as on the box; gsis_set_tile and
 * gsis_autotune return GSIS_ESTATE (as do gsis_gsis_correct and
 * gsis_precondition without centroids) and gsis_batch_create GSIS_EINVAL.  EINVAL when an index, area, normal, volume or centroid is
 * invalid (a face whose centroid distance along its normal is not
 * positive), a cell has more than 16 faces or is not closed (its area times
 * outward normals do not sum to zero within 1e-9 of its area), the faces
 * have more than 32 distinct orientations up to sign, the nodes fall into
 * more than 256 classes, or a class's upwind graph has a cycle (a mesh no
 * sweep orders exactly); ESTATE out of order. */
gsis_status gsis_set_spatial_mesh(gsis_ctx *ctx, int ncell, const double *volume, int nface, const int *face_cell,
                                  const double *face_geom, const double *cell_center, const double *face_center);

/* Boundary condition of slot face (GSIS_FACE_*): kind GSIS_DIFFUSE_WALL with
 * wall velocity u and temperature T (rho ignored; the wall density is set so
 * the discrete mass flux is zero), or GSIS_MAXWELL_INFLOW with the Maxwellian
 * (rho, u, T) entering through the face (Tr = T for the diatomic VDF).  Must
 * precede gsis_bind_workspace. */
gsis_status gsis_set_boundary(gsis_ctx *ctx, int face, int kind, const double u[3], double T, double rho);

/* Boundary flux of the macroscopic correction (Sec. 3.3, Eq. G13_VDF and
 * Eq. GSIS-DVM-flux).  At every boundary face the correction's flux is the
 * kinetic flux of f^{n+1/2} plus the change, from W^{n+1/2} to the iterate
 * W^m, of a model flux: the half-range flux of the cell's distributions with
 * the face's boundary rule (incoming wall Maxwellian at zero net mass flux,
 * or the inflow).  GSIS_WALLFLUX_MAXWELL (the default): the cell's Maxwellian
 * (f1 = (dr/2) Tr M).  GSIS_WALLFLUX_G13: its Grad-13 distributions, in
 * velocities of sqrt(2 R T0)
 *   f0 = M [1 + sigma:cc / (rho Tt^2) + 2 (q.c) / (rho Tt^2) (2 |c|^2 / (5 Tt) - 1)],
 *   f1 = (dr/2) Tr f0 + 2 M (qr.c) / (rho Tt),
 * c = xi - u, M the Maxwellian of (rho, u, Tt), built from the iterate's
 * rho, u, Tt, Tr and the stress and heat fluxes of Eq. (full_constitutive) at
 * the cell: the NSF values of the iterate's central gradients (one-sided next
 * to a non-fluid neighbour; on an unstructured mesh the least-squares
 * gradients of u, Tt and Tr) plus the cell's high-order terms, the kinetic
 * values of f^{n+1/2} minus the NSF values at W^{n+1/2}.  Either way the flux
 * at W^{n+1/2} is the kinetic one, so a kinetic fixed point stays a fixed
 * point.  Must precede gsis_bind_workspace; EINVAL on an unknown model,
 * ESTATE once bound. */
gsis_status gsis_set_wall_flux(gsis_ctx *ctx, int model);

/* Bytes of device workspace the context needs (after the mask is set). */
gsis_status gsis_workspace_size(const gsis_ctx *ctx, size_t *bytes);

/* Bind caller-owned device memory (>= gsis_workspace_size bytes, 256-byte
 * aligned) and upload the geometry and boundary tables.  Synchronises. */
gsis_status gsis_bind_workspace(gsis_ctx *ctx, void *device_ptr, size_t bytes);

/* HIP stream (hipStream_t) for all later device work; NULL = null stream. */
gsis_status gsis_set_stream(gsis_ctx *ctx, void *hip_stream);

/* f0 = M(rho, u, T), f1 = (dr/2) Tr M in every fluid cell; resets the
 * residual snapshot and the pass counter.  Asynchronous. */
gsis_status gsis_init_maxwellian(gsis_ctx *ctx, double rho, const double u[3], double T, double Tr);

/* npasses kinetic passes (Algorithm 3 with one exact upwind solve per pass):
 * reference distribution, boundary values from f^n, implicit upwind sweep in
 * place, moment reduction.  Asynchronous. */
gsis_status gsis_kinetic_step(gsis_ctx *ctx, int npasses);

/* Cell moments of the current state, [ncell][GSIS_NMOM_*] FP64 (NaN in solid
 * cells), to host memory (synchronises) or device memory (asynchronous). */
gsis_status gsis_moments(gsis_ctx *ctx, double *out, int out_is_device);

/* GSIS-II macroscopic correction (Algorithm 2, Sec. 3.3): inner_iters >= 0
 * point-Jacobi iterations of the synthetic equations with the high-order
 * terms of Eq. (full_constitutive) and the boundary flux of gsis_set_wall_flux,
 * then the update of Eq. (updatef), whose moments are applied at once and
 * whose pointwise part is deferred until the VDF is next read.  Needs a
 * kinetic step since init.  Asynchronous. */
gsis_status gsis_gsis_correct(gsis_ctx *ctx, int inner_iters);

/* Initial field of Alg. 1, line 1: macro_steps iterations of the macroscopic
 * solver of gsis_gsis_correct with the Euler constitutive relations (no
 * stress, heat flux or HoT; no diffusive term in the pseudo-time diagonal; the
 * boundary faces take the flux of the iterate's own Maxwellian, whichever
 * gsis_set_wall_flux model is set, since without stress and heat flux the
 * Grad-13 distributions are that Maxwellian), started from
 * the current moments; the VDF is corrected to the result as in Eq. (updatef);
 * then kinetic_steps kinetic passes.  Typically after gsis_init_maxwellian,
 * with 1000 and 10.  Asynchronous; EINVAL for negative counts, ESTATE before
 * initialisation. */
gsis_status gsis_precondition(gsis_ctx *ctx, int macro_steps, int kinetic_steps);

/* Convergence criterion of Sec. 5, Eq. (convergence_critertion): volume-weighted
 * relative L2 change of rho, |u| as a vector and Tt since the previous call or
 * init, into eps[3].  A denominator at or below its noise floor gives the
 * absolute change instead: zero for rho and Tt; for u, (1e3 eps)^2 times the
 * sum of Tt^2, eps the unit roundoff of the VDF precision (the velocity of a
 * gas at rest is rounding noise).  Synchronises.  Returns GSIS_ENOTFINITE if a
 * kernel met a non-positive/non-finite density or temperature, and
 * GSIS_EDIVERGED if a component exceeds 1e6 times its reference, the first
 * value of that component computed against a denominator above the floor. */
gsis_status gsis_residual(gsis_ctx *ctx, double eps[3]);

/* Allocation-free variant of gsis_residual, for callers that cannot allocate
 * device memory at all (HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): same result, bit for bit, but the partial sums of its
 * reduction live in a static device array of the library instead of the
 * context's workspace, and the call allocates nothing (no hipMalloc, no
 * events: it is not phase-timed).  The array holds the partial sums of at most
 * 4096 blocks of 256 cells, so contexts of more than 1,048,576 cells get
 * GSIS_EINVAL (checked before anything else).  One array per GPU, shared by
 * every call on that GPU: calls that overlap on one GPU (other streams or host
 * threads) race; the context's device must be the current one. */
gsis_status gsis_residual_noalloc(gsis_ctx *ctx, double eps[3]);

/* Copy the VDF(s) out / in, canonical [cell][node] FP64 in device memory
 * (f1 may be NULL for monatomic).  set_vdf resets the residual snapshot.
 * Asynchronous. */
gsis_status gsis_get_vdf(gsis_ctx *ctx, double *f0_device, double *f1_device);
gsis_status gsis_set_vdf(gsis_ctx *ctx, const double *f0_device, const double *f1_device);

/* Checkpoint: the complete iteration state (VDF, moments, pending correction,
 * residual snapshot, pass counter) as an opaque blob in device memory.
 * Restoring it and continuing is bitwise identical to never stopping.
 * Synchronises. */
gsis_status gsis_state_size(const gsis_ctx *ctx, size_t *bytes);
gsis_status gsis_get_state(gsis_ctx *ctx, void *dst_device);
gsis_status gsis_set_state(gsis_ctx *ctx, const void *src_device);

/* Sweep tile (cells per tile along x, y, z in the octant's upwind frame) and
 * threads per block (64, 128 or 256); all zeros pick the built-in default for the
 * VDF precision.  Only compiled (tx, ty) are accepted (see gsis_tile_shapes). */
gsis_status gsis_set_tile(gsis_ctx *ctx, int tx, int ty, int tz, int block);

/* Current sweep configuration (tx, ty, tz, block) into tile[4]. */
gsis_status gsis_get_tile(const gsis_ctx *ctx, int *tile);

/* Autotuner: performs the next kinetic pass, running its sweep reps >= 1 times
 * under every compiled (tx, ty) tile shape, tile depths tz in {tx/2, tx, 2 tx}
 * and blocks of 128 and 256 threads, timed with HIP events; selects the
 * fastest configuration for the context.  Valid because every configuration
 * gives a bitwise-identical sweep; requires source iteration (inv_dt = 0)
 * and order 1, where the sweep does not read f^n (an order-2 context takes
 * the tile found for its first-order twin through gsis_set_tile).  Writes up to max entries of
 * (tx, ty, tz, block) to cfg_out[4*k] and their mean sweep time in ms to
 * ms_out[k], and the number of entries to *count (any output may be NULL).
 * Synchronises. */
gsis_status gsis_autotune(gsis_ctx *ctx, int reps, int *cfg_out, double *ms_out, int max, int *count);

/* Compiled sweep tile shapes: writes up to max triples (tx, ty, precision in
 * bits: 32 or 64) to out and their number to *count. */
gsis_status gsis_tile_shapes(int *out, int max, int *count);

/* Copy the VDF at nnodes canonical node indices (host array) for every cell,
 * out_device[k][cell] FP64 (f1 of the diatomic gas is not included).  Applies
 * a pending GSIS update first.  Asynchronous. */
gsis_status gsis_get_vdf_nodes(gsis_ctx *ctx, const int *nodes, int nnodes, double *out_device);

/* Phase timing with HIP events on the bound stream.  Phases: */
enum { GSIS_PHASE_PREP = 0,      /* per-cell parameters and boundary densities */
       GSIS_PHASE_SWEEP = 1,     /* implicit upwind sweep (all tile-plane launches of a pass) */
       GSIS_PHASE_MOMENTS = 2,   /* moment reduction and central moments */
       GSIS_PHASE_MACRO = 3,     /* gsis_correct: macroscopic solve and moment update */
       GSIS_PHASE_RESIDUAL = 4,  /* gsis_residual */
       GSIS_PHASE_RECON = 5,     /* order 2: limiter and second-order right-hand side of a pass */
       GSIS_NPHASE = 6 };
/* enable != 0 starts recording (events are created on first use and kept by the
 * context); 0 stops. */
gsis_status gsis_profile_enable(gsis_ctx *ctx, int enable);
/* Synchronises, then returns the accumulated milliseconds and call counts per
 * phase (arrays of GSIS_NPHASE); reset != 0 clears them. */
gsis_status gsis_profile_read(gsis_ctx *ctx, double *ms, long long *calls, int reset);

/* Number of kinetic passes since init/set_vdf. */
gsis_status gsis_pass_count(const gsis_ctx *ctx, long long *passes);

/* NUL-terminated message of the last error on ctx (static string if ctx is NULL). */
const char *gsis_last_error(const gsis_ctx *ctx);

/* ------------------------------------------------------------------ batches
 * Many independent problems of Algorithm 1 -- cavities of uneven cell counts,
 * velocity grids and gas parameters -- iterated together: every kernel launch
 * of a GSIS iteration (kinetic pass, GSIS-II correction, residual) covers all
 * cases at once through a per-launch table of (case, block) pairs, the sweep
 * runs one launch per global tile hyperplane across all cases, and the
 * iteration is captured once into a HIP graph and replayed.
 *
 * The cases are contexts made with gsis_create and configured as usual (mask,
 * boundaries) but NOT bound: the batch binds them all inside one caller-owned
 * workspace.  They must share vdf_dtype and species and use inv_dt = 0
 * (source iteration) and order 1.  The batch borrows the contexts: destroy it before
 * them, and do not bind them elsewhere.  Once bound, each context also works
 * on its own (gsis_moments, gsis_get_vdf, gsis_residual, ...) on the batch's
 * stream.  One tile shape (tx, ty, tz, block) serves every case. */
typedef struct gsis_batch gsis_batch;

/* ncases in 1..4096 distinct, unbound contexts (host array).  EINVAL if they
 * differ in precision or gas, or have inv_dt != 0, order 2 or a velocity node
 * list. */
gsis_status gsis_batch_create(gsis_batch **out, gsis_ctx *const *cases, int ncases);
gsis_status gsis_batch_destroy(gsis_batch *b);
/* Bytes of device memory the batch needs (all cases plus launch tables and
 * residual history). */
gsis_status gsis_batch_workspace_size(gsis_batch *b, size_t *bytes);
/* Carve the workspace (256-byte aligned, caller owned) into every case and
 * upload the launch tables.  Synchronises. */
gsis_status gsis_batch_bind_workspace(gsis_batch *b, void *device_ptr, size_t bytes);
/* Stream of all batch work and of its contexts; graph capture needs a
 * non-null stream. */
gsis_status gsis_batch_set_stream(gsis_batch *b, void *hip_stream);
/* One tile shape for every case (see gsis_set_tile); all zeros = default. */
gsis_status gsis_batch_set_tile(gsis_batch *b, int tx, int ty, int tz, int block);
gsis_status gsis_batch_get_tile(const gsis_batch *b, int *tile);
/* Time the batched sweep of the next pass under every compiled tile
 * configuration (reps timed launches after a warm-up) and keep the fastest;
 * counts as one kinetic pass of every case.  Same output as gsis_autotune.
 * Synchronises. */
gsis_status gsis_batch_autotune(gsis_batch *b, int reps, int *cfg_out, double *ms_out, int max, int *count);
/* gsis_init_maxwellian on every case; clears the residual history. */
gsis_status gsis_batch_init_maxwellian(gsis_batch *b, double rho, const double u[3], double T, double Tr);
/* iters GSIS iterations of every case, each: one kinetic pass,
 * gsis_gsis_correct(inner_iters) (skipped when inner_iters == 0), and the
 * residual of Sec. 5 against the previous iteration, recorded in the history.
 * use_graph != 0 captures one iteration into a HIP graph (kept and reused
 * while inner_iters and the tile shape stay the same) and replays it iters
 * times; 0 launches the kernels directly.  Asynchronous. */
gsis_status gsis_batch_run(gsis_batch *b, int iters, int inner_iters, int use_graph);
/* Residual history since init: eps[it][case][3] (rho, |u|, Tt) for the last
 * min(count, capacity) iterations, oldest first; *count = iterations returned
 * (at most max).  Synchronises; ENOTFINITE if any case flagged a non-positive
 * or non-finite state. */
gsis_status gsis_batch_residuals(gsis_batch *b, double *eps, int max, int *count);
/* Milliseconds of device time of the last gsis_batch_run (events around it). */
gsis_status gsis_batch_last_run_ms(gsis_batch *b, double *ms);
const char *gsis_batch_last_error(const gsis_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* GSIS_H */
