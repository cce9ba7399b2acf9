/*
 * dvm.h -- C ABI of libdvm_hip.so, the MI355X (gfx950) implementation of the
 * iterative discrete-velocity scheme for the steady Shakhov model equation
 * (Zhu, Wang, Chen, Guo, Zhang, "GPU acceleration of an iterative scheme for
 * gas-kinetic model equations with memory reduction techniques",
 * arXiv:1810.00348).
 *
 * One outer iteration n -> n+1 (Sec. 2.2, eq. "iter_outer"):
 *   1. per cell, from the conserved moments W^n = (rho, rho U, rho E) and the
 *      heat flux q^n (eq. "mom"): U, T, the relaxation rate 1/tau
 *      (tau = mu/p, viscosity law and mu_ref of Sec. 4, eq. "mu_ref"), the
 *      parameters of the Shakhov equilibrium f^S (eq. "feq") and of its
 *      conservative correction (discrete mass, momentum and energy of the
 *      corrected equilibrium equal those of f, computed in FP64);
 *   2. for every discrete velocity, the first-order upwind implicit sweep
 *      along its characteristic direction (eq. "sweeping_example"), with the
 *      equilibrium evaluated on the fly, never stored;
 *   3. the discrete moments of the new f (eq. "macros"), accumulated in FP64,
 *      the wall densities from the non-penetration condition
 *      (eqs. "maxwell_wall", "rho_wall"), the total-mass rescaling of a
 *      closed domain (Sec. 3.4) and the relative change of the conserved
 *      fields (Sec. 4.1).
 *
 * Units: lengths in units of the reference length that defines Kn,
 * velocities in units of sqrt(2 R T0), temperature in T0, density in rho0.
 *
 * Conventions
 *   - Cell index c = i + nx*(j + ny*k); field arrays are structure-of-arrays
 *     FP64 (a 3-vector field u is u[d*N + c]).
 *   - Host arrays are owned by the caller; every call that reads or writes
 *     them copies synchronously on the context's stream.
 *   - Device memory: a context allocates none.  The caller (the Python
 *     binding uses torch) allocates a workspace of dvm_required_workspace()
 *     bytes and lends it with dvm_bind_workspace(); the library never frees
 *     it.  The workspace must stay alive and untouched until dvm_destroy().
 *     Small contexts may instead take the library's static workspace
 *     (dvm_bind_static_workspace).  Only the self-test
 *     dvm_selftest_wave_reduce allocates (and frees) device memory.
 *   - Every call returns a dvm_status; on an error the context keeps the
 *     last good iterate and dvm_last_error() describes the failure.
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - Call order: dvm_create -> dvm_set_face_bc / dvm_set_solid /
 *     dvm_set_closed -> dvm_required_workspace -> dvm_bind_workspace ->
 *     dvm_init_uniform | dvm_init_fields | dvm_set_state -> dvm_iterate ...
 *
 * Against the interface planned for this library the calls differ in
 * these ways: dvm_set_solid_mask is also available as dvm_set_solid (the
 * same call); dvm_init_fields takes the target total mass (double, 0 = keep
 * the given density) where an integer flag normalised to the unit mass;
 * dvm_get_state / dvm_set_state also carry M0, the reference mass of the
 * closed-domain rescaling, so that a resumed run continues bit for bit;
 * dvm_create takes the precision as int (a dvm_precision value) so that the
 * ABI does not depend on the size of an enum; and the calls after
 * dvm_set_velocity_groups (schedule, streams, parameter precision, the
 * static workspace, stress, launch timings) are additions.
 */
#ifndef DVM_H
#define DVM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dvm_ctx dvm_ctx;

typedef enum {
    DVM_OK = 0,
    DVM_NOT_CONVERGED = 1,   /* max_iters reached before the tolerance      */
    DVM_ERR_ARG = -1,        /* invalid argument                           */
    DVM_ERR_STATE = -2,      /* call out of order                          */
    DVM_ERR_OOM = -3,        /* workspace too small / host allocation      */
    DVM_ERR_DEVICE = -4,     /* HIP runtime error                          */
    DVM_ERR_NONPHYSICAL = -5 /* rho <= 0, T <= 0 or NaN                     */
} dvm_status;

typedef enum { DVM_F64 = 0, DVM_F32 = 1 } dvm_precision;

/* boundary kinds of a box face */
typedef enum {
    DVM_BC_WALL = 0,     /* Maxwell diffuse wall (eqs. "maxwell_wall", "rho_wall") */
    DVM_BC_FREE = 1,     /* particles entering get the free-stream equilibrium   */
    DVM_BC_SPECULAR = 2  /* symmetry plane (z- face only, even velocity count)   */
} dvm_bc_kind;

typedef struct { int nx, ny, nz; double lx, ly, lz; } dvm_grid;       /* uniform cells */
typedef struct { int m[3]; double vmax[3]; } dvm_vgrid;                /* m[d] >= 2 uniform nodes
                                                                          on [-vmax, vmax], both
                                                                          ends included, trapezoid
                                                                          weights (Sec. 4.1)      */
typedef struct {
    double kn;      /* Knudsen number: tau(rho=1,T=1) = kn*15 sqrt(pi)/((5-2w)(7-2w)) */
    double omega;   /* viscosity index, mu ~ T^omega (0.81 for argon, Sec. 4)        */
    double pr;      /* Prandtl number of the Shakhov model (2/3); pr = 1 gives BGK   */
    int conservative_correction;  /* 1 (default): corrected equilibrium            */
} dvm_gas;

typedef struct {
    int kind;       /* dvm_bc_kind                                                   */
    double u[3];    /* wall or free-stream velocity                                  */
    double T;       /* wall or free-stream temperature                               */
    double rho;     /* free-stream density (DVM_BC_FREE only)                        */
} dvm_face_bc;

typedef struct {
    int nx, ny, nz, ncells, nfluid;
    int m[3], nvel;
    int precision;              /* dvm_precision                                  */
    int brick[3];               /* cells per brick of the sweep schedule          */
    int vel_per_lane;           /* discrete velocities handled by one lane        */
    int tiles_per_octant;       /* 64-lane velocity tiles per octant              */
    int sweep_launches;         /* sweep kernel launches per iteration            */
    size_t workspace_bytes;
    int pipelined;              /* sweep body: 0 plain, 1 software-pipelined, 2
                                   pipelined in one dependency-driven launch       */
    int velocity_groups;        /* velocity groups swept one after another        */
    int parameter_bits;         /* 64: per-cell parameters, Gaussian tables and
                                   equilibrium evaluation in FP64; 32: in FP32    */
    int sweep_streams;          /* streams the per-diagonal sweep launches use    */
} dvm_info;

/* Create a context.  precision: DVM_F64 or DVM_F32, the storage and update
   type of f.  With DVM_F32 the sweep also evaluates the equilibrium in FP32:
   the per-cell parameters (U, T, 1/tau, the Shakhov coefficients and the
   multipliers of the conservative correction) are computed in FP64 from the
   FP64 conserved moments and then rounded to FP32 for the sweep, so the
   FP32 collision operator conserves mass, momentum and energy to FP32
   rounding; the velocity moments are accumulated in FP64, and the
   finalisation, wall densities, mass rescaling and residual are FP64 in
   both precisions.  hip_stream:
   a hipStream_t on which every kernel and copy is issued (NULL = null stream).
   Defaults: all six faces diffuse walls at rest with T = 1, no solid, closed.
   Errors: DVM_ERR_ARG for non-positive sizes, lengths, kn, pr or T. */
dvm_status dvm_create(const dvm_grid* grid, const dvm_vgrid* vgrid, const dvm_gas* gas,
                      int precision, void* hip_stream, dvm_ctx** out);

/* Boundary condition of box face 0..5 = x-, x+, y-, y+, z-, z+.  Errors:
   DVM_ERR_ARG (bad face/kind, T <= 0, specular on a face other than z- or
   with an odd velocity count along z), DVM_ERR_STATE after binding. */
dvm_status dvm_set_face_bc(dvm_ctx* ctx, int face, const dvm_face_bc* bc);

/* Solid cells (mask[c] != 0, nx*ny*nz bytes, host, copied by the call)
   inside the box; their faces are diffuse walls with velocity u_wall and
   temperature T_wall (the solid body of the cube flow, Sec. 4.2).  mask may
   be NULL (no solid).  Before binding the workspace (DVM_ERR_STATE after
   it); DVM_ERR_ARG for T_wall <= 0. */
dvm_status dvm_set_solid(dvm_ctx* ctx, const unsigned char* mask, const double u_wall[3],
                         double T_wall);
/* The same call under the name of the solid-mask setter. */
dvm_status dvm_set_solid_mask(dvm_ctx* ctx, const unsigned char* mask, const double u_wall[3],
                              double T_wall);

/* closed != 0: rescale the density field after every iteration so that the
   total mass stays that of the initial state (Sec. 3.4, internal flows). */
dvm_status dvm_set_closed(dvm_ctx* ctx, int closed);

/* Non-uniform tensor-product mesh (the stretched meshes of the paper's cube
   runs, Sec. 4.2): cell sizes along x (nx values), y (ny) and z (nz), host
   arrays copied by the call; NULL keeps that axis uniform (length / n).
   Each axis's sizes must be positive and sum to its length in dvm_grid
   (relative 1e-9).  The upwind coefficient of a cell along d is
   |xi_d| / h_d(cell) (finite-volume flux form) and cell volumes weigh the
   total mass.  Before binding the workspace; DVM_ERR_STATE after it,
   DVM_ERR_ARG for bad sizes, or with the ES-BGK model where the velocity
   set leaves 1 velocity per lane (the mesh is then left as it was). */
dvm_status dvm_set_spacing(dvm_ctx* ctx, const double* hx, const double* hy, const double* hz);

/* Collision model: 0 Shakhov (default; Sec. 2.1), 1 ES-BGK -- the scheme
   applies to other model equations too (Sec. 2.1).  ES-BGK target: the
   Gaussian G = rho (2 pi)^{-3/2} det(Lam)^{-1/2} exp(-c^T Lam^{-1} c / 2)
   with Lam = (T/2) I / Pr + (1 - 1/Pr) Theta (normalised units, R T = T/2),
   Theta the stress per unit mass of the iterate (kept as state, computed
   with the other moments about U^{n+1}), relaxation frequency Pr p / mu,
   the same conservative correction.  Needs Pr >= 2/3 (Lam positive
   definite); on a stretched mesh (dvm_set_spacing, in either order) a
   velocity set that fills 2 or more velocities per lane (DVM_ERR_ARG
   otherwise, the previous model kept).  The sweep has one cross factor
   exp(-(A_xy cx cy + A_xz cx cz + A_yz cy cz)) per phase-space point
   more, the parameter pass one pass over the velocity set per cell.  The stress starts (dvm_init_*) and restarts (dvm_set_state) at
   the equilibrium (T/2) I of the state.  Before binding the workspace
   (DVM_ERR_STATE after it); DVM_ERR_ARG otherwise. */
dvm_status dvm_set_model(dvm_ctx* ctx, int model);

/* ES-BGK: the stress per unit mass of the current iterate, 6 x ncells
   doubles (xx, yy, zz, xy, xz, yz), into a host array.  DVM_ERR_STATE for
   the Shakhov model or before an initial state. */
dvm_status dvm_get_stress(dvm_ctx* ctx, double* stress);

/* ES-BGK: replace the stress of the current iterate (same layout; after
   dvm_init_* or dvm_set_state, which reset it to the equilibrium), e.g. to
   carry a state over between FP32 and FP64 contexts.  DVM_ERR_STATE for the
   Shakhov model or before a state; DVM_ERR_ARG for non-finite values. */
dvm_status dvm_set_stress(dvm_ctx* ctx, const double* stress);

/* Velocity nodes and quadrature weights per axis (m[d] values each, host
   arrays copied by the call) in place of the uniform trapezoid axes -- the
   non-uniform velocity grids the paper recommends over very large uniform
   ones (Sec. 5.2).  NULL nodes and weights keep that axis uniform on
   [-vmax, vmax].  Nodes must increase and be symmetric about 0
   (xi[M-1-a] = -xi[a], relative 1e-12; the sweep splits each axis at 0),
   weights positive and symmetric.  Equilibria, emission shapes and moments
   then use these nodes and weights.  Before binding the workspace
   (DVM_ERR_STATE after it); DVM_ERR_ARG for invalid axes. */
dvm_status dvm_set_velocity_axes(dvm_ctx* ctx, const double* xi_x, const double* w_x, const double* xi_y,
                                 const double* w_y, const double* xi_z, const double* w_z);

/* Spatial order of the upwind sweep: 1 (default; the paper's first-order
   scheme, Sec. 2.2) or 2 (the extension its closing section proposes, from
   three consecutive cells along each axis).  Second order: every face
   carries the upwind cell's value extrapolated linearly from that cell and
   its own upwind neighbour, f + (f - f_up)/2 (f alone when that cell's
   upwind side is a boundary); a boundary face carries its inflow value; a
   symmetry plane is an interior face whose far side is the mirror image;
   the wall densities are balanced with what crosses the wall faces.  On a
   stretched mesh the extrapolation follows the straight line through the
   two cell centres, f + theta (f - f_up) with theta = h / (h + h_up) along
   that axis, and the sweep takes the pipelined body with 2 or more
   velocities per lane (a schedule without one fails at binding).  Before
   binding the workspace (DVM_ERR_STATE after it); DVM_ERR_ARG for another
   order.  Order 2 doubles the face and mirror-plane buffers and the
   sweep's LDS plane. */
dvm_status dvm_set_order(dvm_ctx* ctx, int order);

/* Sweep the velocity set in `groups` parts, one after another, within each
   iteration: each octant's 64-lane velocity tiles are split into `groups`
   consecutive ranges of (nearly) equal size (at most one range per tile).
   The sweep of one velocity does not depend on the others within an
   iteration (the equilibrium and the wall densities come from the previous
   iterate, Sec. 2.2 and 3.4), so the result is that of one group up to the
   order of the FP64 moment sums.  The face buffers, the mirror planes of a
   specular side and the per-tile moment partials then hold one range only,
   which divides the workspace (dominated by them on large grids) by about
   `groups`; an FP64 accumulator of 8 x 16 doubles per cell is added when
   groups > 1.  This is how the largest meshes of Sec. 4.2 (181 x 181 x 191
   cells, 48^3 velocities) fit one device.  Before binding the workspace;
   DVM_ERR_STATE after it, DVM_ERR_ARG for groups < 1. */
dvm_status dvm_set_velocity_groups(dvm_ctx* ctx, int groups);

/* Sweep schedule in place of the library's choice, for measurements and
   tests of a particular kernel: vel_per_lane discrete velocities per lane
   (1, 2, 4 or 8), bricks of bx x by x bz cells, body 1 = plain,
   2 = software-pipelined, 3 = software-pipelined in one dependency-driven
   launch per velocity group and specular phase (first-order Shakhov sweep
   only): the waves take bricks from a device-wide counter in diagonal order
   and start each one as soon as its three upwind bricks have published,
   instead of one launch per brick diagonal; a wait that does not end
   within half a second fails the iteration with DVM_ERR_DEVICE (the
   iterate is not updated).  0 keeps the library's choice for that value
   (the brick's x and y sizes default to those of the chosen velocities per
   lane).  The result is the same for every schedule up to the order of the
   FP64 moment sums; only the speed differs.  The brick column is shortened
   where the sweep's 32-bit face offsets would overflow (dvm_get_info
   reports the schedule in use).  DVM_ERR_ARG for values out of range or a
   kernel shape that is not built for the context's precision, mesh kind,
   order and model (the previous schedule stays; a later dvm_set_order,
   dvm_set_model or dvm_set_spacing that leaves the request without a
   kernel makes dvm_bind_workspace fail with DVM_ERR_ARG).  Before binding
   the workspace (DVM_ERR_STATE after it). */
dvm_status dvm_set_schedule(dvm_ctx* ctx, int vel_per_lane, int bx, int by, int bz, int body);

/* FP32 contexts: bits = 64 keeps the per-cell parameters (U, 1/tau, the
   Shakhov coefficients, the conservative-correction multipliers), the
   Gaussian factor tables and the evaluation of the equilibrium in FP64; f
   is still stored and updated in FP32 and takes the equilibrium rounded
   once.  bits = 32 (default): all of them in FP32 (see dvm_create).  Built
   for the first-order Shakhov sweep on a uniform mesh with 4 velocities per
   lane, 4x2 bricks and a pipelined body; otherwise dvm_bind_workspace fails
   with DVM_ERR_ARG.  FP64 contexts accept 64 only.  Before binding the
   workspace (DVM_ERR_STATE after it). */
dvm_status dvm_set_parameter_precision(dvm_ctx* ctx, int bits);

/* Streams for the per-diagonal sweep launches (1, 2, 4 or 8; default 2).
   The octants of a phase (all eight, or the four of one side of a
   specular plane) are split into that many sets, each set's launches go to
   a stream of its own, forked from the context's stream after the
   parameters and joined back before the moments are finalised: the octants
   do not depend on each other within an iteration, so a set's next
   diagonal fills the device while another set's launch drains.  The result
   is the same for every count.  The streams (default priority) and their
   events are created at the first iteration that needs them; a count above
   the one created then is refused with DVM_ERR_STATE. */
dvm_status dvm_set_sweep_streams(dvm_ctx* ctx, int streams);

/* Bytes of device workspace the context needs with its current settings. */
dvm_status dvm_required_workspace(dvm_ctx* ctx, size_t* bytes);

/* Lend the workspace (device pointer, >= required bytes, 256-byte aligned).
   Uploads the velocity set and boundary tables and computes the wall
   emission shapes on the device. */
dvm_status dvm_bind_workspace(dvm_ctx* ctx, void* device_ptr, size_t bytes);

/* For callers that cannot allocate device memory (code that runs under HIP
   graph capture, tight serving loops, hosts that forbid hipMalloc): bind the
   library's own static workspace of the current device instead of a lent
   one.  That workspace is a file-scope device array of 64 MiB per device
   (DVM_STATIC_WORKSPACE_BYTES), held by each device the library runs on
   until the process ends; this call allocates nothing.  It holds contexts
   whose dvm_required_workspace() is at most that size (e.g. 16^3 cells x
   12^3 velocities FP64 needs 35 MiB); larger ones get DVM_ERR_OOM, nothing
   changed.  One device array serves one context at a time: binding it to a
   new context takes it from the previous one, whose later calls that touch
   the workspace (init, iterate, get/set state, fields, stress) return
   DVM_ERR_STATE; calls of two contexts on one device that overlap in time
   race on the array.  Everything a kernel reads before writing is written
   by this call or the initial state, so the previous contents do not
   matter.  The current device must be the stream's device (DVM_ERR_ARG
   otherwise).  Other errors as dvm_bind_workspace. */
#define DVM_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
dvm_status dvm_bind_static_workspace(dvm_ctx* ctx);

/* Uniform initial state (rho, u, T); q = 0; wall densities from the
   non-penetration flux of the initial equilibrium (Sec. 2.2, initial
   equilibrium from uniform macroscopic fields). */
dvm_status dvm_init_uniform(dvm_ctx* ctx, double rho, const double u[3], double T);

/* Initial state from host fields rho[N], u[3N], T[N] (solid cells ignored).
   target_mass > 0: rho is first scaled so that sum(rho) dV = target_mass.
   Errors: DVM_ERR_NONPHYSICAL if a fluid cell has rho <= 0, T <= 0 or a
   non-finite value. */
dvm_status dvm_init_fields(dvm_ctx* ctx, const double* rho, const double* u, const double* T,
                           double target_mass);

/* Run up to max_iters outer iterations, stopping after the first one whose
   residual is <= tol (tol <= 0: run exactly max_iters).  Residual: the max
   over rho, rho Ux, rho Uy, rho Uz, rho E of ||phi^{n+1}-phi^n||_2 /
   ||phi^{n+1}||_2 over fluid cells.  iters_done, residual may be NULL.
   Returns DVM_OK (converged or tol <= 0), DVM_NOT_CONVERGED, or an error
   (DVM_ERR_NONPHYSICAL leaves the last good iterate in place). */
dvm_status dvm_iterate(dvm_ctx* ctx, int max_iters, double tol, int* iters_done,
                       double* residual);

/* Residual of each conserved field after the last iteration (5 values). */
dvm_status dvm_get_residuals(dvm_ctx* ctx, double r[5]);

/* Macroscopic fields of the current iterate: rho[N], u[3N], T[N], q[3N]
   (any may be NULL); solid cells get 0. */
dvm_status dvm_get_fields(dvm_ctx* ctx, double* rho, double* u, double* T, double* q);

/* Checkpoint / resume: W[5N] (rho, rho U, rho E), q[3N], rho_w[6N] (wall
   density of each cell face, side-major), M0 (total mass of the initial
   state).  Any pointer may be NULL on get. */
dvm_status dvm_get_state(dvm_ctx* ctx, double* W, double* q, double* rho_w, double* M0);
dvm_status dvm_set_state(dvm_ctx* ctx, const double* W, const double* q, const double* rho_w,
                         double M0);

/* Sizes and schedule of the context. */
dvm_status dvm_get_info(dvm_ctx* ctx, dvm_info* info);

/* Per-phase device timing.  enable = 1 records HIP events around the
   parameter, sweep and finalisation phases of every following iteration
   (on the context's stream; the sweep phase from the fork of its streams to
   their join).  enable = 2 also records events around every sweep launch on
   the stream it is issued to.  dvm_get_timings returns the accumulated
   milliseconds and the number of timed iterations, dvm_get_launch_timings
   the summed duration of the timed sweep launches and their number; each
   resets what it returns.  DVM_ERR_ARG for another level. */
dvm_status dvm_set_timing(dvm_ctx* ctx, int enable);
dvm_status dvm_get_timings(dvm_ctx* ctx, double* ms_params, double* ms_sweep,
                           double* ms_finalize, int* iterations);
dvm_status dvm_get_launch_timings(dvm_ctx* ctx, double* ms_total, long long* launches);

/* Check of the wave-level 13-moment reduction used by the sweep kernel:
   in[64*13] (lane-major: in[lane*13 + k]) -> out[13] = sum over lanes. */
dvm_status dvm_selftest_wave_reduce(const double* in, double* out);

/* Message of the last error on the calling thread ("" if none). */
const char* dvm_last_error(void);

/* Release the context (not the borrowed workspace). */
void dvm_destroy(dvm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* DVM_H */
