/*
 * lgs_lbm.h -- C ABI of the MI355X liquid-gas-solid lattice Boltzmann library.
 *
 * One call of lbm_step advances every lattice instance of a context by one
 * time step of the method of Bogner & Ruede, "Liquid-gas-solid flows with
 * lattice Boltzmann: Simulation of floating bodies":
 *
 *   1. body remap          (Sec. 2.3 cell-centre mapping; Sec. 2.4 conversions
 *                           into / out of obstacle on B(x))       -- if a body moved
 *   2. stream + collide    (Sec. 2.1 Eq. stream and the collide step with the
 *                           force term of Eq. forceterm; Sec. 2.2 mass exchange
 *                           and Eq. reconstruct; Sec. 2.3 Eq. noslip), fused with
 *      momentum exchange   (Eqs. momentumexchange, momentuminterface, netforce,
 *                           torque) on the same pass
 *   3. interface conversions (Sec. 2.2, thresholds -eps / 1+eps)
 *
 * Units are lattice units (cell size 1, time step 1).  Cell (x, y, z) spans
 * [x, x+1] x [y, y+1] x [z, z+1]; its centre is (x+.5, y+.5, z+.5) (Sec. 2.1).
 * Faces that are not periodic are static no-slip walls just outside the
 * lattice (halfway bounce-back).
 *
 * Host arrays exchanged through lbm_read_fields / lbm_write_fields are laid
 * out x fastest: scalars [nz][ny][nx], populations [19][nz][ny][nx] in the
 * D3Q19 order of the paper's Fig. d3q19 caption: C, W, E, N, S, T, B, TW, TE,
 * TN, TS, NW, NE, SW, SE, BW, BE, BN, BS (E = +x, N = +y, T = +z).  Flags are
 * one byte per cell: bits 0-1 type (0 gas, 1 liquid, 2 interface,
 * 3 obstacle), bits 2-5 owning body of an obstacle cell.
 *
 * Every function returns an int32 status (LBM_OK = 0, negative on error) and
 * leaves its outputs untouched on error; lbm_last_error() gives a
 * thread-local message.  No exception crosses the ABI.  A context is used by
 * one host thread; all its device work is ordered on one HIP stream.
 */
#ifndef LGS_LBM_H
#define LGS_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBM_OK = 0,
    LBM_ERR_INVALID = -1,  /* bad argument (message says which)              */
    LBM_ERR_NOMEM = -2,    /* workspace too small or allocation failed       */
    LBM_ERR_DEVICE = -3,   /* a HIP call failed                              */
    LBM_ERR_UNSTABLE = -4, /* non-finite values or a list overflow detected  */
    LBM_ERR_STATE = -5     /* call not valid in the context's current state  */
};

/* Storage of the populations.  All variants store the deviation f_i - w_i
 * from the rest weights (w_i of the caption of Fig. d3q19) and collide in
 * FP32: FP32 stores it as float, FP16 as binary16 scaled by fp16_scale (a
 * power of two), BF16 as bfloat16 unscaled. */
enum { LBM_FP32 = 0, LBM_FP16_DEV = 1, LBM_BF16_DEV = 2 };

enum { LBM_PERIODIC_X = 1, LBM_PERIODIC_Y = 2, LBM_PERIODIC_Z = 4 };

enum {
    LBM_FIELD_POP = 1,   /* f_i (absolute, not the stored deviation), 19 per cell */
    LBM_FIELD_FLAGS = 2, /* one byte per cell (write: bits 0-5 as above)         */
    LBM_FIELD_PHI = 3,   /* fill level phi (Sec. 2.2)                             */
    LBM_FIELD_MASS = 4,  /* liquid mass m of interface cells (Sec. 2.2)           */
    LBM_FIELD_RHO = 5,   /* density sum_i f_i (read only)                         */
    LBM_FIELD_VEL = 6    /* velocity sum_i c_i f_i / rho, 3 per cell [3][z][y][x] (read only) */
};
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_U8 = 2 };

/* Parts of one step, for phase-isolated testing with lbm_step_phases. */
enum { LBM_PHASE_REMAP = 1, LBM_PHASE_SWEEP = 2, LBM_PHASE_CONVERT = 4, LBM_PHASE_ALL = 7 };

/* Gas-side reconstruction set in interface cells (Sec. 2.2, Eq. reconstruct).
 * The normal n = -grad(phi) (central differences over the 6 axis
 * neighbours; liquid 1, gas 0, interface phi, obstacle / wall: own phi)
 * points into the gas; a link i >= 1 counts as "from the gas side" when
 * c_i.n < -1e-3 |n|_1.
 *   0: links with a gas source, plus links from the gas side      (default)
 *   1: links with a gas source only
 *   2: links with a gas source, plus links with c_i.n <= +1e-3 |n|_1
 *      (the printed "c_i^T n <= 0", tangential links included)            */
enum { LBM_RECON_GAS_SIDE = 0, LBM_RECON_GAS_ONLY = 1, LBM_RECON_PAPER_LE = 2 };

#define LBM_MAX_BODIES 16

typedef struct lbm_config {
    int32_t nx, ny, nz;        /* lattice cells                                      */
    int32_t storage;           /* LBM_FP32 / LBM_FP16_DEV / LBM_BF16_DEV              */
    double tau;                /* BGK relaxation time, > 0.5 (Sec. 2.1)                */
    double accel[3];           /* body acceleration a (gravity = {0, 0, -g}) (Eq. forceterm) */
    double rho_gas;            /* gas density rho_G, p_G = rho_G / 3 (Sec. 2.2)        */
    double eps;                /* conversion threshold epsilon (Sec. 2.2), >= 0        */
    double fill_height;        /* H: initial liquid below z = H (cells of fill
                                  clamp(H - z, 0, 1)), hydrostatic density
                                  rho = rho_G - 3 a_z (H - z_c) + noise             */
    double init_ux_surface;    /* u_s: initial u_x = u_s z_c (2H - z_c) / H^2 (0 = rest) */
    uint32_t periodic;         /* LBM_PERIODIC_* bits; other faces are walls          */
    int32_t recon_mode;        /* LBM_RECON_*                                         */
    uint64_t seed;             /* initial density noise: SplitMix64(seed ^ cell index) */
    double noise_amp;          /* noise amplitude A: rho += A (2U - 1)                 */
    double fp16_scale;         /* power of two (FP16 storage); 0 = default 4096        */
    int32_t max_bodies;        /* bodies per instance, 0 .. LBM_MAX_BODIES             */
    int32_t host_body_update;  /* free bodies: 0 = rigid-body update on the device at
                                  the end of every step (no host round trip);
                                  1 = on the host: every step synchronises,
                                  reads the forces and runs lbm_integrate_body */
    double wall_vel[3];        /* velocity of the non-periodic faces: moving no-slip
                                  walls (Eq. noslip with u_w = wall_vel; the paper's
                                  channel is driven by its long sides); 0 = static */
    double surface_tension;    /* sigma >= 0, below 0.1 (Sec. 2.2, Laplace pressure):
                                  interface cells rebuild their gas-side populations
                                  with the gas pressure p_G + 2 sigma kappa, kappa the
                                  mean curvature taken as half the divergence of the
                                  unit surface normals (central differences of the
                                  fill levels, then of the normals of the six axis
                                  neighbours; an obstacle or wall neighbour lends the
                                  cell's own normal).  kappa > 0 where the liquid is
                                  convex (a droplet: 1/R).  0 = no surface tension;
                                  sigma > 0 adds one small kernel over the interface
                                  cells per step and 4 bytes per cell of workspace */
} lbm_config;

/* Body shapes (Sec. 2.3 maps any shape by its cell centres; the paper's
 * experiments use cuboids and spheres). */
enum { LBM_SHAPE_CUBOID = 0, LBM_SHAPE_SPHERE = 1 };

/* A rigid body (Sec. 2.3).  A cell is an obstacle cell of the body iff its
 * centre c satisfies, with d = c - pos (minimum image on periodic axes) and
 * everything in FP64 without fused multiply-add:
 *   cuboid: |R^T d|_k <= half_ext[k] for k = 0..2, R the rotation of `quat`;
 *   sphere: d_x^2 + d_y^2 + d_z^2 <= r^2 (summed in that order), r = half_ext[0].
 * Moving-wall velocity at a point p: vel + omega x (p - pos). */
typedef struct lbm_body {
    double half_ext[3]; /* half extents in the body frame (cells)                  */
    double pos[3];      /* centre of gravity o, lattice coordinates               */
    double quat[4];     /* orientation w, x, y, z (unit)                          */
    double vel[3];      /* world frame, cells per step                            */
    double omega[3];    /* world frame, radians per step                          */
    double density;     /* rho_s relative to the liquid's 1                       */
    uint32_t fixed;     /* 1: the caller holds the pose (moves it only through
                           lbm_set_body); 0: free -- after every full step the
                           update of lbm_integrate_body, fed with the mean of
                           this and the previous step's fluid force and torque,
                           advances it on the DOFs of dof_mask (on the device,
                           same FP64 operations, or on the host: see
                           lbm_config.host_body_update)                          */
    uint32_t dof_mask;  /* free bodies: bits 0-2 translation x,y,z, 3-5 rotation */
    uint32_t shape;     /* LBM_SHAPE_CUBOID (0) or LBM_SHAPE_SPHERE (radius half_ext[0];
                           half_ext[1..2] are ignored)                           */
} lbm_body;

typedef struct lbm_ctx lbm_ctx;

/* Device bytes needed for n_inst instances described by cfgs[0..n_inst-1]. */
int32_t lbm_workspace_size(const lbm_config* cfgs, int32_t n_inst, size_t* bytes);

/* Create a context and initialise every instance (basin of lbm_config, no
 * body yet).  d_workspace: device memory of at least lbm_workspace_size bytes
 * owned by the caller (e.g. a torch uint8 tensor kept alive for the context's
 * lifetime), or NULL to let the library allocate and own it.  hip_stream: the
 * hipStream_t all work is ordered on (NULL = null stream).  Checks: tau > 0.5,
 * max_k n_k |a_k| < 0.1 c_s^2 (the incompressibility bound of Sec. 2.1),
 * storage, sizes, eps >= 0, rho_gas > 0.  Besides the workspace the library
 * allocates one 8-byte word of pinned host memory per instance, where the
 * steps report the highest layer that may hold fluid (the bulk sweep's
 * grid bound); without it the bulk sweep launches every layer. */
int32_t lbm_create(const lbm_config* cfgs, int32_t n_inst, void* d_workspace, size_t ws_bytes, void* hip_stream,
                   lbm_ctx** out);
int32_t lbm_destroy(lbm_ctx* ctx);

/* Set (add or move) body `body` of instance `inst`.  The pose takes effect at
 * the next step's remap phase; the first set of a body maps it (covered liquid
 * mass goes to the ledger).  Checks: body inside the non-periodic extent with
 * one free cell of margin, surface speed < 1 cell per step (Sec. 2.4 assumes
 * obstacles move less than a cell per step), moves by less than one cell
 * since its last mapping, and three free cells between the bounding boxes of
 * two bodies.  Synchronises the stream (reads the device's body records).
 * A free body's previous-step force is forgotten. */
int32_t lbm_set_body(lbm_ctx* ctx, int32_t inst, int32_t body, const lbm_body* b);
/* Current state of a body (free bodies: as the device advanced it).
 * Synchronises the stream. */
int32_t lbm_get_body(lbm_ctx* ctx, int32_t inst, int32_t body, lbm_body* b);

/* Advance all instances by nsteps full steps (remap of moved bodies, sweep,
 * conversions and force reduction, then the device update of free bodies,
 * whose new pose the next step maps).  Asynchronous on the context's stream
 * unless an instance updates its free bodies on the host.  A free-body update
 * that breaks the lbm_set_body checks is rejected (the body keeps its pose):
 * on the device the next lbm_sync returns LBM_ERR_UNSTABLE naming the reason,
 * on the host lbm_step returns it.  Each step's bulk sweep covers the layers
 * up to a bound the host derives from the reports of earlier steps; the host
 * waits for the GPU when it runs further ahead of them than about 4 GB of
 * queued bulk-sweep traffic (2 to 8 steps). */
int32_t lbm_step(lbm_ctx* ctx, int32_t nsteps);

/* One step restricted to the phases in phase_mask (LBM_PHASE_*), for tests.
 * LBM_PHASE_CONVERT without LBM_PHASE_SWEEP first scans for the interface
 * cells past the thresholds. */
int32_t lbm_step_phases(lbm_ctx* ctx, int32_t phase_mask);

/* Fluid-on-body force and torque about the body's centre, world frame, of the
 * last completed sweep (FP64 sums).  Synchronises the stream. */
int32_t lbm_body_forces(lbm_ctx* ctx, int32_t inst, int32_t body, double force[3], double torque[3]);

/* Copy a field of one instance to / from host memory (synchronous).
 * bytes must equal cells * components * sizeof(dtype).  POP is the absolute
 * f_i; gas and obstacle cells hold unspecified populations.  Writing FLAGS
 * takes the written obstacle cells as the mapping of the bodies already set,
 * at their current poses (an obstacle cell of a body that is not set is an
 * error), and no remap follows until a body moves or is set again: to have
 * the library map a body onto written fields, set it after writing them. */
int32_t lbm_read_fields(lbm_ctx* ctx, int32_t inst, int32_t field, int32_t dtype, void* host_dst, size_t bytes);
int32_t lbm_write_fields(lbm_ctx* ctx, int32_t inst, int32_t field, int32_t dtype, const void* host_src,
                         size_t bytes);

/* Liquid mass sum_LIQ rho + sum_IF m (FP64 reduction on the device in a
 * fixed order: one partial per 4096 cells, then their sum, so the result
 * does not depend on scheduling) and the ledger: mass added to the fluid
 * minus mass removed by remaps and undistributable conversion excess.  total - ledger is conserved up to
 * round-off and moving-wall mass fluxes.  Synchronises. */
int32_t lbm_mass_total(lbm_ctx* ctx, int32_t inst, double* total, double* ledger);
int32_t lbm_set_ledger(lbm_ctx* ctx, int32_t inst, double ledger);

/* lbm_mass_total without any use of the context's workspace or of device
 * memory allocation, for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * kernels and same result bit for bit; the partial sums (one per 4096 cells)
 * and the result live in a static device array of the library, 16384
 * partials + 1 double (128 KiB) per GPU, kept until the process ends.
 * Lattices of more than 16384 * 4096 = 67,108,864 cells: LBM_ERR_INVALID
 * (use lbm_mass_total).  Every call on a GPU shares that array: calls that
 * overlap on one GPU (several host threads, or streams of several contexts)
 * race.  Synchronises. */
int32_t lbm_mass_total_noalloc(lbm_ctx* ctx, int32_t inst, double* total, double* ledger);

/* Counts of the last conversion phase: filled, emptied, gas->interface,
 * liquid->interface.  Synchronises. */
int32_t lbm_conversion_counts(lbm_ctx* ctx, int32_t inst, int64_t counts[4]);

/* Number of liquid cells with a gas neighbour (0 for a closed interface
 * layer, Sec. 2.2).  Synchronises. */
int32_t lbm_liq_gas_contacts(lbm_ctx* ctx, int32_t inst, int64_t* contacts);

/* Wait for all work of the context, then report what the device flagged:
 * LBM_ERR_UNSTABLE for a non-finite or non-positive density, a rejected
 * free-body update or a list overflow; LBM_ERR_DEVICE if a bulk sweep's
 * layer bound missed a layer holding fluid (an internal error). */
int32_t lbm_sync(lbm_ctx* ctx);

/* Kernel timing: while enabled, HIP start / stop events are attached to the
 * dispatches of the two sweep kernels of every step (extended launch on the
 * context's stream: the events time the kernel itself, not marker packets
 * around it).  lbm_kernel_time returns the summed
 * duration in milliseconds and the number of timed steps since the last
 * enable (synchronises).  Kernel ids: 0 = bulk sweep (liquid cells whose
 * sources are fluid or static wall), 1 = boundary sweep (interface cells and
 * liquid cells next to gas or a body), 2 = both. */
int32_t lbm_enable_kernel_timing(lbm_ctx* ctx, int32_t enable);
int32_t lbm_kernel_time(lbm_ctx* ctx, int32_t kernel, double* total_ms, int64_t* launches);

/* Launch configuration of a context (not a quantity of the method).
 * tile_x: width along x of the bulk-sweep tiles, 32, 64 or 128 cells
 * (256 / tile_x rows), or 0: tiles of 256 consecutive cells of a z-layer
 * (rows packed end to end; every lane holds a cell for widths that are not
 * a multiple of the tile width).  batched: step all instances with one launch per
 * kernel (all instances must share one storage type; no effect with one
 * instance; the default for several instances of one storage type).
 * use_graph: lbm_step replays pairs of full steps from a captured HIP graph
 * when no instance updates free bodies on the host; the capture is redone
 * when the step parity or the set of instances that remap changes.
 * stream_store: 1 = the bulk sweep writes the populations with
 * non-temporal (streaming) stores that pass the caches: faster once the
 * populations a step moves (both lattices over the layers up to the bulk
 * sweep's layer bound) exceed the 256 MiB cache in front of HBM, slower
 * below it (the default follows that size).
 * boundary_layout: work layout of the boundary sweep (interface cells and
 * liquid cells next to gas or a body): 0 = 8 lanes per cell, the links
 * shared through LDS (short lists); 1 = one thread per cell (long lists,
 * coalesced loads).  Both compute the same rules.
 * Synchronises.  Errors: LBM_ERR_INVALID for a bad width or flag, or mixed
 * storage in a batch. */
int32_t lbm_set_tuning(lbm_ctx* ctx, int32_t tile_x, int32_t batched, int32_t use_graph, int32_t stream_store,
                       int32_t boundary_layout);
int32_t lbm_get_tuning(lbm_ctx* ctx, int32_t* tile_x, int32_t* batched, int32_t* use_graph, int32_t* stream_store,
                       int32_t* boundary_layout);

/* Autotuner.  First the bulk sweep: reps launches on the current state for
 * every tile width (32, 64, 128, and 0: packed rows) and store policy
 * (cached, and streaming where a step's populations exceed the 256 MiB
 * cache; below it the trials, which sweep one cached source, would favour
 * streaming stores), the fastest kept.  Then the boundary sweep: reps launches with each
 * work layout, the faster kept (skipped, layout unchanged and boundary_ms
 * -1, when the device has no room for a copy of the interface cells' mass,
 * flags and counters, 9 bytes per cell).  The state does not change: the
 * sweeps write the lattice the next step overwrites, the boundary sweep's
 * in-place updates are undone from that copy after every launch, and the
 * boundary-list count is reset.  Outputs (nullable): the chosen width, store
 * policy and layout, and the average launch times in ms.  Synchronises.
 * reps: 1..64. */
int32_t lbm_autotune(lbm_ctx* ctx, int32_t reps, int32_t* tile_x, int32_t* stream_store, int32_t* boundary_layout,
                     double* bulk_ms, double* boundary_ms);

/* Number of cells the last sweep of an instance handled in the boundary
 * kernel (synchronises). */
int32_t lbm_boundary_cells(lbm_ctx* ctx, int32_t inst, int64_t* n);

/* Rigid-body update on the host (the paper couples to a rigid-body engine;
 * this is a plain semi-implicit Euler step, dt = 1), for callers that move
 * held bodies themselves: mass M = density * 8 hx hy hz (cuboid) or
 * density * 4/3 pi r^3 (sphere), V += (F + M a) / M on translational DOFs
 * (dof_mask bits 0-2), Omega += I_SS^-1 T_S on rotational DOFs S (bits 3-5; I
 * the world-frame inertia about the centre: cuboid M/3 (h_j^2 + h_k^2) on the
 * body axes, sphere 2/5 M r^2), pos += V, quat rotated by Omega. */
int32_t lbm_integrate_body(const lbm_body* in, const double force[3], const double torque[3],
                           const double accel[3], uint32_t dof_mask, lbm_body* out);

const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LGS_LBM_H */
