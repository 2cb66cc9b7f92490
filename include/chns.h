/*
 * chns.h -- C ABI of the MI355X (gfx950) time-step library for the two-phase
 * Cahn-Hilliard Navier-Stokes (CHNS) model of Khanwale et al., "A fully-coupled
 * framework for solving Cahn-Hilliard Navier-Stokes equations: second-order,
 * energy-stable numerical methods on adaptive octree based meshes"
 * (arXiv 2009.06628).
 *
 * Model (paper, governing-equations section): phase field phi in [-1, 1],
 * chemical potential mu = psi'(phi) - Cn^2 lap(phi) with psi = (phi^2-1)^2/4,
 * mixture density rho = alpha phi + beta and viscosity eta = gamma phi + xi
 * built from the pulled-back phi* = clamp(phi, -1, 1) (remark on the
 * pull-back), thermodynamically consistent flux
 * J = (rho_- - rho_+)/(2 rho_+ Cn) grad mu, momentum with the Korteweg
 * stress, pressure (1/We) grad p, viscosity (1/Re) div(eta grad v) and
 * gravity rho g_hat / Fr with g_hat = (0,-1,0), solenoidal velocity.
 * Non-dimensional groups Pe, Re, We, Cn, Fr as defined there; mobility 1.
 *
 * Discretisation (a split step on a uniform MAC grid; the paper's own
 * Crank-Nicolson / FEM / Newton layout is not used): the library advances
 *   S1  explicit CH stage with the advective flux u A(phi),
 *   S2  (I - dt kM S L + dt kM Cn^2 L L) phihat = r, kM = 1/(Pe Cn), S = stabiliser,
 *   S3  mu^{n+1} = psi'(phi^n) + S (phihat - phi^n) - Cn^2 L phihat,
 *   S4  phi^{n+1} = phi^n - dt D(u A(phi^n) - kM G mu^{n+1})  (mass conserving),
 *   S5  J = -(alpha/Cn) G mu^{n+1},  m = A(alpha phi^n + beta) u^n + J / Pe,
 *   S6  rho^{n+1}, eta^{n+1} from clamp(phi^{n+1}),
 *   S7  per axis a:  (rho_f^{n+1}/dt) u*_a - (1/Re) div(eta grad u*_a)
 *         = ((rho_f^{n+1}+rho_f^n)/(2dt)) u_a^n - N_a(m, u^n)
 *           - (1/(We Cn)) A_a(phi^n) G_a mu^{n+1} + rho_f^{n+1} g_hat_a / Fr,
 *       N_a the skew-symmetric advection of the appendix remark,
 *   S8  -D(rho_f^{-1} G p) = -(We/dt) D u*,  mean(p) = 0,
 *   S9  u^{n+1} = u* - (dt/We) rho_f^{-1} G p.
 * The variable-coefficient systems (S7, S8) are solved matrix-free by
 * multigrid-preconditioned conjugate gradients on the device.  The S2
 * system has constant coefficients: on a single grid whose axes all have at
 * most 2048 cells it is solved directly (the 1D second difference of each
 * axis is diagonalised by an orthonormal DCT-II basis on a walled axis and
 * the real Fourier basis on a periodic one; the solve is one transform per
 * axis, a division by 1 - a lam + b lam^2, and the inverse transforms, in
 * FP64 on the grid's stream: a radix-2 FFT along periodic axes of 16 .. 512
 * cells (a power of two), a product with the dense basis along the others).
 * chns_set_option(g, CHNS_OPT_CH_SOLVER, CHNS_CH_PCG) selects
 * multigrid-preconditioned CG for S2 instead; larger grids and 3D batches
 * always use it.
 *
 * Three-phase model (nphases = 3; the paper is two-phase, this extends its
 * binary free-energy density by the Boyer-Lapuerta construction): phases
 * i = 1, 2, 3 with volume fractions c_i = (1 + phi_i)/2, sum_i c_i = 1; the
 * state holds phi_1, phi_2 and phase 3 is implied.  Free energy
 * (1/Cn) sum_i (Sigma_i/2) int psi(phi_i) + Cn^2/2 |grad phi_i|^2 with the
 * spreading coefficients Sigma_i = sigma_ij + sigma_ik - sigma_jk; the
 * constrained potentials mu~_i = psi'(phi_i) - Cn^2 lap phi_i - w_i Lambda,
 * Lambda = sum_j psi'(phi_j), w_i = Sigma_T/(3 Sigma_i),
 * 3/Sigma_T = sum_j 1/Sigma_j, sum to zero; every phase follows the paper's
 * CH equation d phi_i/dt + div(u phi_i) = kM lap mu~_i; rho and eta are
 * sum_i rho_i c_i*, sum_i eta_i c_i* with c_i* = clamp(c_i, 0, 1); the
 * consistent flux is J = -(kM/2) sum_i rho_i grad mu~_i and the capillary
 * force -(1/(2 Cn)) sum_i Sigma_i phi_i grad mu~_i.  The step T1..T9 is
 * S1..S9 per phase with Lambda taken at t^n (two S2 solves).  For a pair
 * i|j with the third phase absent it is the two-phase step with
 * 1/We = sigma_ij.
 *
 * Data layout (device memory, float64, row-major, x fastest):
 *   cell arrays   idx = i + nx*(j + ny*k), nx*ny*nz entries (nz = 1 in 2D);
 *   face arrays   one per axis a, same shape as the cell arrays; entry c is
 *                 the face between cell c - e_a and cell c.  On a walled axis
 *                 the entry with index 0 along that axis is the wall face
 *                 (its normal velocity is 0) and the opposite wall face is
 *                 not stored.
 *
 * Ownership: every device array (state, workspace) belongs to the caller.
 * The library keeps raw pointers and small host metadata, never allocates
 * device memory, and runs all work on the stream given at creation.  Handles
 * are not thread-safe; distinct handles are independent.
 *
 * Errors: functions return CHNS_OK (0), the warning CHNS_ENOCONV (> 0: the
 * call completed but a linear solve stopped at max_iter), or a negative code.
 * After a negative code the outputs of that call are unspecified.
 * chns_last_error() returns a message for the most recent failure on the
 * calling thread.
 */
#ifndef CHNS_H
#define CHNS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CHNS_OK = 0,
    CHNS_ENOCONV = 1,      /* warning: a solve hit max_iter; see stats      */
    CHNS_EINVAL = -1,      /* bad argument or unsupported grid              */
    CHNS_ENOMEM = -2,      /* workspace smaller than chns_workspace_size    */
    CHNS_EDEVICE = -3,     /* HIP runtime error (message in last_error)     */
    CHNS_ENONFINITE = -4   /* NaN / Inf detected in a residual              */
};

enum { CHNS_BC_PERIODIC = 0, CHNS_BC_WALL = 1 };
enum { CHNS_FP64 = 0, CHNS_FP32_REFINE = 1 };

/* Grid description.  dim = 2 or 3; n[a] cells along axis a (n[2] ignored in
 * 2D); h the uniform cell size; bc[a] per axis: periodic, or no-slip /
 * no-flux walls on both ends (paper: boundary conditions of the
 * mass-conservation proposition).  precision selects the arithmetic of the
 * linear solves (CHNS_FP64, or FP64 conjugate gradients preconditioned by
 * FP32 multigrid: vectors, operator apply, updates, dot products and the
 * coarsest inverse in FP64; coefficients, sweeps and transfers of the
 * V-cycle in FP32).  nphases = 2 (the paper's two-phase model) or 3 (three-phase
 * model, see below; single grids only -- the batched and adjoint entry
 * points reject it).
 * Supported sizes: every n[a] >= 2 and even, and repeated halving of all axes
 * while they stay even must reach a grid of at most 512 cells.            */
typedef struct {
    int dim;
    int n[3];
    double h;
    int bc[3];
    int precision;
    int nphases;
} chns_grid_desc;

/* Physical and numerical parameters (non-dimensional; the phi = +1 fluid is
 * the reference, rho_+ = eta_+ = 1).  inv_Fr = 1/Fr, 0 disables gravity.
 * dt the time step, S the CH stabiliser (S >= 1 keeps the CH sub-step energy
 * stable for |phi| <= 1).  rtol_* are relative residual tolerances
 * ||b - Ax||_2 <= rtol ||b||_2 of the CH, momentum and pressure solves;
 * max_iter caps every PCG solve.                                         */
typedef struct {
    double rho_minus, eta_minus;
    double Re, We, Cn, Pe, inv_Fr;
    double dt, S;
    double rtol_ch, rtol_mom, rtol_p;
    int max_iter;
    int reserved;
    /* three-phase grids (nphases = 3) only: densities and viscosities of
     * phases 1, 2, 3 (relative to the reference fluid), pairwise surface
     * tensions (sigma_12, sigma_13, sigma_23) with every spreading
     * coefficient sigma_ij + sigma_ik - sigma_jk > 0.  rho_minus and
     * eta_minus are then unused, and We only scales the pressure (the
     * capillary forces come from sigma_ij).                               */
    double rho3[3], eta3[3], sigma3[3];
} chns_props;

/* Caller-owned device pointers of the state.  phi, p, mu: cell arrays;
 * u[a]: face arrays (u[2] unused in 2D).  chns_step reads phi, u, p and
 * overwrites them with the new state; mu receives mu^{n+1}.
 * Three-phase grids: phi and phi2 hold phi_1 = 2 c_1 - 1 and
 * phi_2 = 2 c_2 - 1 (phase 3 is implied: c_3 = 1 - c_1 - c_2), and mu, mu2
 * receive the constrained chemical potentials mu~_1, mu~_2.  phi2 and mu2
 * are ignored on two-phase grids.                                        */
typedef struct {
    void *phi;
    void *u[3];
    void *p;
    void *mu;
    void *phi2;
    void *mu2;
} chns_state;

/* Host-side statistics of the last step of a chns_step call.            */
typedef struct {
    int iters_ch, iters_mom[3], iters_p;
    int unconverged;            /* bit 0: CH, bits 1..3: momentum, bit 4: p */
    double res_ch, res_mom[3], res_p;   /* final relative residuals        */
    double mass_plus, mass_minus;       /* sum (1 +- phi)/2 h^d            */
    double energy;                      /* discrete total energy           */
    double umax, divmax;                /* max |u|, max |D u|              */
    double mass_phase[3];               /* sum c_i h^d of phases 1, 2, 3
                                           (two-phase grids: mass_plus,
                                           mass_minus, 0)                   */
} chns_step_stats;

typedef struct {
    int iters;
    double rel_res;
} chns_solve_stats;

/* Bytes of device workspace that chns_create_grid needs for this grid
 * (field buffers, multigrid hierarchy, coarse-grid inverse, reduction
 * scratch, and the S2 bases: n_a^2 + n_a doubles per axis when every axis
 * has at most 2048 cells).  Returns CHNS_EINVAL for an unsupported
 * description.                                                           */
int chns_workspace_size(const chns_grid_desc *desc, size_t *bytes);

/* Create a handle.  workspace: device memory of at least
 * chns_workspace_size bytes, 256-byte aligned, owned by the caller and kept
 * alive until chns_destroy_grid.  hip_stream: a hipStream_t (NULL = default
 * stream).  No device memory is allocated here or later; the S2 bases are
 * built on the host and copied into the workspace here (synchronously).
 * The handle also creates dim - 1 non-blocking streams of default priority
 * for the velocity components 1 .. dim-1 (their momentum solves of S7
 * overlap with the first component's) and one more for the set-up of the
 * S8 coefficients and pressure hierarchy, which needs only phi^{n+1} and
 * runs during those solves; event waits order all of them with hip_stream,
 * so every call still completes on hip_stream.  chns_destroy_grid releases
 * them.  A handle must not be used by two host
 * threads at once.                                                       */
int chns_create_grid(const chns_grid_desc *desc, void *workspace, size_t bytes,
                     void *hip_stream, struct chns_grid **out);

/* Set / change the parameters (host struct, copied).  Must be called before
 * the first chns_step.  Rebuilds the constant CH multigrid hierarchy.     */
int chns_set_properties(struct chns_grid *g, const chns_props *props);

/* Advance the state nsteps time steps (S1..S9 each) in place on the grid's
 * stream.  If stats is not NULL the call synchronises the stream and fills
 * it (solver statistics of the last step, diagnostics of the final state).
 * The momentum solves of the components and the pressure set-up run on
 * their own streams, driven by host worker threads of the handle (created
 * on its first such step, joined by chns_destroy_grid; serially on the
 * grid's stream while per-kernel timing is on, or with the option
 * CHNS_OPT_SERIAL_COMPONENTS set); the results do not depend on which.
 * Returns CHNS_ENOCONV if any solve of any step hit max_iter.            */
int chns_step(struct chns_grid *g, chns_state *st, int nsteps, chns_step_stats *stats);

/* Energy-law monitor of one step (the time-step condition of the paper's
 * energy-stability theorem), with the step's own fields u^{n+1}, mu^{n+1},
 * eta^{n+1} in place of the theorem's Crank-Nicolson averages:
 *   visc   (1/Re) ||sqrt(eta) grad u||^2: sum_a u_a^T K_a u_a h^d with K_a
 *          the viscous part of the step's momentum operator of component a
 *   chem   (1/(Pe Cn^2 We)) ||G mu||^2
 *   cubic  (1/(24 We Cn)) sum 6 max(|phi^n|, |phi^{n+1}|) |phi^{n+1} - phi^n|^3 h^d,
 *          a bound of the magnitude of the theorem's cubic term (the third
 *          derivative of psi is 6 phi, taken between phi^n and phi^{n+1})
 *   inert  (1/8) sum_a sum_faces |A_a(rho^{n+1} - rho^n)| (u_a^{n+1} - u_a^n)^2 h^d,
 *          a bound of the magnitude of the density-change term
 *   holds  dt (visc + chem) >= cubic + inert (the theorem's condition with
 *          the bounds: the energy cannot rise)
 *   dt_max dt sqrt(dt (visc + chem) / (cubic + inert)): the bounds grow like
 *          dt^3 and the dissipation like dt (HUGE_VAL when both bounds are 0)
 *   energy_before, energy_after: the discrete total energy at t^n, t^{n+1}. */
typedef struct {
    double visc, chem, cubic, inert;
    double dt_max;
    double energy_before, energy_after;
    int holds;
    int reserved;
} chns_energy_monitor;

/* One step (chns_step with nsteps = 1) that also evaluates the energy-law
 * monitor on the device (one reduction kernel between S8 and S9, plus the
 * energy of the state before and after).  Two-phase grids only
 * (CHNS_EINVAL otherwise).  Synchronises the stream.  Return codes as
 * chns_step.                                                              */
int chns_step_monitor(struct chns_grid *g, chns_state *st, chns_energy_monitor *out);

/* Stand-alone pressure solve of S8:  -D(rho_f^{-1} G p) = rhs, mean(p) = 0,
 * with rho a cell array of densities (rho_f = face averages, used as is)
 * and rhs a cell array (projected to mean zero internally; not modified).
 * p (cell array) is the initial guess on entry and the solution on exit.  */
int chns_solve_pressure(struct chns_grid *g, const void *rho, const void *rhs, void *p,
                        double rtol, int max_iter, chns_solve_stats *stats);

/* Apply the pressure operator of S8: y = -D(rho_f^{-1} G x) with rho_f the
 * face averages of the cell density rho (no pull-back).  x, y: cell arrays.
 * Synchronises the stream.  Used to check the stencil kernel on its own.  */
int chns_apply_pressure_operator(struct chns_grid *g, const void *rho, const void *x, void *y);

/* ---- discrete adjoint -------------------------------------------------
 * Reverse-mode derivative of one call of the step map S1..S9 (the split
 * scheme of the paper's time discretisation, including the pull-back of phi
 * in the density and viscosity maps, the consistent flux J and the
 * potential-form surface tension), for losses of the final phi and u.
 * The adjoint needs its own workspace (caller-owned device memory, 256-byte
 * aligned, size from chns_adjoint_workspace_size), attached once per handle.
 */
int chns_adjoint_workspace_size(const chns_grid_desc *desc, size_t *bytes);
int chns_attach_adjoint_workspace(struct chns_grid *g, void *workspace, size_t bytes);

/* Adjoint variables: device pointers with the state's layout (phi a cell
 * array, u[a] face arrays; u[2] unused in 2D).  Entries of u on wall faces
 * are ignored on input and written as 0.                                   */
typedef struct {
    void *phi;
    void *u[3];
} chns_adj;

/* One reverse step.  fwd: the state (phi^k, u^k, and p^{k-1}, the pressure
 * initial guess the forward step used) at the start of forward step k; it
 * is read only: the call recomputes S1..S8 of that step into the adjoint
 * workspace.  lam_in: dL/d(phi^{k+1}, u^{k+1}); lam_out receives
 * dL/d(phi^k, u^k).  lam_out may be the same arrays as lam_in (in place),
 * but must not otherwise overlap them or fwd.  The three adjoint elliptic
 * solves (pressure, momentum per component, CH) use the forward operators,
 * which are symmetric, with the forward tolerances.  If grad_params (host,
 * 2 doubles) is not NULL it ACCUMULATES this step's parameter derivatives:
 * grad_params[0] += dL/dsigma, grad_params[1] += dL/dM, for the surface
 * tension sigma = 1/We and the mobility M = We/Pe at fixed Re, Cn, ratios
 * (so k_M = 1/(Pe Cn) = M sigma / Cn; u^{k+1} does not depend on We through
 * the projection); this synchronises the stream.  Returns CHNS_ENOCONV if a
 * forward or adjoint solve hit max_iter.                                   */
int chns_adjoint_step(struct chns_grid *g, const chns_state *fwd, const chns_adj *lam_in, chns_adj *lam_out,
                      double grad_params[2]);

/* The forward fields of one step that its reverse step reads (device arrays
 * of the grid's layout, caller-owned): phihat (S2), phi_new = phi^{n+1}
 * (S4), mu = mu^{n+1} (S3), p = p^{n+1} (S8) in cell arrays, ustar[a] = u*
 * (S7) in the face arrays of component a (ustar[2] NULL in 2D).          */
typedef struct {
    void *phihat, *phi_new, *mu, *p;
    void *ustar[3];
} chns_record;

/* chns_step with nsteps = 1 that also copies the step's forward fields into
 * rec (for chns_adjoint_step_recorded; checkpointed reverse passes that
 * re-run a segment record its steps instead of recomputing them again in
 * every reverse step).  Same return codes as chns_step.                    */
int chns_step_record(struct chns_grid *g, chns_state *st, const chns_record *rec);

/* chns_adjoint_step with the forward fields of the step taken from rec,
 * written by chns_step_record from the state fwd under the same properties,
 * instead of recomputing S1..S8 (fwd->p is not read).  The step's forward
 * fields are a function of fwd alone (every solve starts from a guess built
 * from fwd), so the result equals chns_adjoint_step's bit for bit.
 * Argument rules, accumulation into grad_params and return codes as for
 * chns_adjoint_step.                                                      */
int chns_adjoint_step_recorded(struct chns_grid *g, const chns_state *fwd, const chns_record *rec,
                               const chns_adj *lam_in, chns_adj *lam_out, double grad_params[2]);

/* ---- batched ensemble -------------------------------------------------
 * Many independent problems of uneven size (same dim and precision) advanced
 * together: one persistent kernel per time step in which each workgroup
 * takes whole problems from a longest-first queue and runs S1..S9 for them,
 * with the solver loops on the device.  nsteps launches can be captured once
 * into a hipGraph and replayed.  The state of all problems is packed back to
 * back: problem i occupies cells [offsets[i], offsets[i+1]) of each packed
 * array (its own layout inside, as for a single grid).                    */
struct chns_batch;

/* Per-problem statistics of one chns_batch_step call.                    */
typedef struct {
    int iters_ch, iters_mom[3], iters_p;  /* last step                              */
    int flags;        /* OR over the call: bit 0 CH, bits 1..3 momentum, bit 4
                         pressure unconverged; bit 5 non-finite residual        */
    int steps;        /* steps taken in the call                                */
    int pad;
    long long total_iters;               /* PCG iterations of all solves       */
    double res_ch, res_mom[3], res_p;    /* last step's relative residuals     */
} chns_batch_stats;

/* Two forms of the batched step:
 *  CHNS_BATCH_PERSISTENT  one persistent kernel per step; each workgroup
 *                         takes whole problems (largest first) and runs S1..S9
 *                         with its solver loops on the device;
 *  CHNS_BATCH_TILED       one launch per sweep over the cells of all problems,
 *                         cut into tiles of tile_cells cells (a 256-thread
 *                         workgroup per tile); per-problem solver scalars, the
 *                         small multigrid levels one workgroup per problem.  A
 *                         captured (graph) step launches a fixed number of CG
 *                         iterations per solve (the budgets); eager steps run
 *                         every solve to convergence with host checks.       */
enum { CHNS_BATCH_PERSISTENT = 0, CHNS_BATCH_TILED = 1 };

#define CHNS_MAX_TUNING 16
/* Autotuner result: the chosen form, its launch shape (persistent: block
 * threads per workgroup, grid workgroups; tiled: tile_cells) and time per
 * step, the graph iteration budgets, and every candidate that was timed
 * (cand_block holds tile_cells for tiled candidates).                     */
typedef struct {
    int mode, block, grid, tile_cells;
    double ms_per_step;
    int budget_ch, budget_mom, budget_p;
    int ncand;
    int cand_mode[CHNS_MAX_TUNING], cand_block[CHNS_MAX_TUNING], cand_grid[CHNS_MAX_TUNING];
    double cand_ms[CHNS_MAX_TUNING];
} chns_batch_tuning;

/* Workspace bytes for count problems (descs[i] as for a single grid),
 * including, for 2D batches, the S2 bases of every distinct problem shape
 * and per-problem pointer tables of the direct solve.                    */
int chns_batch_workspace_size(int count, const chns_grid_desc *descs, size_t *bytes);

/* Create a batch: descs[count], props[count] (copied), caller-owned device
 * workspace (256-byte aligned).  hip_stream: the caller's stream; the batch
 * runs on an internal non-blocking stream ordered after it and before any
 * later work on it.  Builds the constant CH hierarchies (synchronises).
 * 2D batches solve S2 directly, as single grids do: the problems of one
 * shape share their bases, and each solve is four batched transform
 * launches per shape plus a scaling launch.  Both forms (persistent,
 * tiled) use it.  3D batches and axes over 2048 cells keep
 * multigrid-preconditioned CG for S2.  No device
 * memory is allocated here or later.                                      */
int chns_create_batch(int count, const chns_grid_desc *descs, const chns_props *props, void *workspace,
                      size_t bytes, void *hip_stream, struct chns_batch **out);

/* Packed-layout offsets (count + 1 entries, in cells; host array).       */
int chns_batch_offsets(struct chns_batch *b, long long *offsets);

/* Advance every problem nsteps steps in place.  packed: device pointers to
 * the packed arrays.  use_graph != 0 captures the nsteps launches into a
 * hipGraph on the first call and replays it while nsteps, the pointers and
 * the launch shape stay the same.  stats (host, count entries) or NULL; if
 * given the call synchronises and returns CHNS_ENOCONV / CHNS_ENONFINITE
 * when any problem's solve reported it.  In the tiled form a captured step
 * launches a fixed number of iterations per solve (the budgets): such a call
 * keeps a copy of the state and always synchronises; when a solve ran out of
 * its budget, that solve's budgets grow (iterations by max(2, a quarter),
 * the FP32 refinement round by max(2, a half), at most to the largest
 * max_iter), the state is restored and the steps are captured and replayed
 * again, so the result is that of converged solves.  Grown budgets stay for
 * later calls.  A graph holds at most 20 steps; longer calls replay a graph
 * of the largest divisor of nsteps up to 20.                              */
int chns_batch_step(struct chns_batch *b, const chns_state *packed, int nsteps, int use_graph,
                    chns_batch_stats *stats);

/* Persistent form with block threads per workgroup (64..512, multiple of
 * 64) and grid persistent workgroups (>= 1).                              */
int chns_batch_set_launch(struct chns_batch *b, int block, int grid);

/* Tiled form with tile_cells cells per tile (multiple of 256; uploads the
 * tile lists, synchronous).                                               */
int chns_batch_set_tiled(struct chns_batch *b, int tile_cells);

/* CG iterations a captured tiled step launches per solve (CH, each momentum
 * component, pressure); a problem that needs more is reported unconverged.
 * The autotuner sets them from the iterations it observed.               */
int chns_batch_set_budget(struct chns_batch *b, int iters_ch, int iters_mom, int iters_p);

/* Time steps_per_trial steps for each candidate form and launch shape, keep
 * the fastest, set the graph budgets, and restore the packed state
 * (bitwise) afterwards.  Synchronises.  result (host) may be NULL.        */
int chns_batch_autotune(struct chns_batch *b, const chns_state *packed, int steps_per_trial,
                        chns_batch_tuning *result);

/* Release the batch (host metadata, stream, events, graph).               */
int chns_destroy_batch(struct chns_batch *b);

/* Per-kernel timing.  chns_set_timing(g, 1) creates a host-side pool of
 * hipEvents (no device memory), resets the counters and makes every later
 * chns_step / chns_solve_pressure bracket each kernel launch with an event
 * pair; chns_set_timing(g, 0) stops it.  chns_get_timing copies one record
 * per kernel class that ran (at most max records; *count receives the number
 * of classes): launches, summed kernel time in ms (hipEventElapsedTime) and
 * summed algorithmic bytes (each array a launch reads or writes counted
 * once).  Timing adds host work per launch; measure throughput without it. */
typedef struct {
    char name[24];
    int launches;
    double ms;
    double bytes;
} chns_kernel_timing;

int chns_set_timing(struct chns_grid *g, int enable);
int chns_get_timing(struct chns_grid *g, chns_kernel_timing *out, int max, int *count);

/* ---- pressure solve without allocation ---------------------------------
 * For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * stand-alone S8 solve of chns_solve_pressure (same operator, kernels,
 * arguments and results), on a grid given by its description instead of a
 * handle, with no workspace argument.  Its multigrid hierarchy, CG vectors
 * and reduction scratch live in a device array of the library of
 * CHNS_NOALLOC_SCRATCH_BYTES bytes, which every GPU the library runs on
 * holds until the process ends; the call allocates nothing (no hipMalloc,
 * no library allocation).  Grids whose solver storage exceeds that size are
 * rejected with CHNS_EINVAL (FP64 needs about 115 bytes per cell plus the
 * coarsest inverse, the precision form about 156: the 256 x 512 grid fits).
 * rho, rhs: cell arrays (device, float64; rhs projected to mean zero
 * internally, not modified); p: initial guess on entry, solution with mean
 * zero on exit.  desc->precision selects FP64 or FP64 CG with the FP32
 * multigrid preconditioner; desc->nphases is ignored.  Runs on hip_stream (NULL: the
 * default stream) and synchronises it before returning.  Every call on a
 * GPU shares that GPU's array and leaves its contents behind: calls that
 * overlap on one GPU (from several threads or streams) race and must be
 * serialised by the caller.  Returns as chns_solve_pressure.              */
#define CHNS_NOALLOC_SCRATCH_BYTES (32u << 20)
int chns_solve_pressure_noalloc(const chns_grid_desc *desc, const void *rho, const void *rhs, void *p,
                                double rtol, int max_iter, void *hip_stream, chns_solve_stats *stats);
/* Size in bytes of that array (CHNS_NOALLOC_SCRATCH_BYTES).              */
size_t chns_solve_pressure_noalloc_capacity(void);

/* Walls with inhomogeneous Dirichlet data (the moving lid of the paper's
 * lid-driven cavity): the wall of walled axis `axis` on side `side` (0: the
 * lower wall, 1: the upper one) moves tangentially with velocity component
 * `component` (!= axis) given by `values`, a face array of that component
 * (device, float64, caller-owned, read by every later step until replaced)
 * whose layer next to the wall (index 0 along `axis` for side 0, n - 1 for
 * side 1) holds the wall speed at the faces' positions on the wall; other
 * entries are not read.  NULL makes that wall component rest again.  The
 * no-slip ghost value next to the wall becomes 2 U - u, so the wall edge of
 * those momentum rows adds 2 k U to their right-hand side (k the edge's
 * viscous coefficient); the normal velocity and the mass and phase fluxes
 * through every wall stay zero.  chns_step_monitor rejects grids with
 * moving walls.                                                            */
int chns_set_wall_velocity(struct chns_grid *g, int axis, int side, int component, const void *values);

/* Per-handle options (host state; take effect from the next call):
 *   CHNS_OPT_CH_SOLVER          CHNS_CH_DIRECT (default where every axis has
 *                               at most 2048 cells: the direct S2 solve),
 *                               CHNS_CH_DIRECT_DENSE (the direct solve with
 *                               the dense basis product on every axis, no
 *                               FFT) or CHNS_CH_PCG (multigrid-preconditioned
 *                               CG); CHNS_EINVAL for DIRECT on larger grids;
 *   CHNS_OPT_SERIAL_COMPONENTS  1: the momentum components of S7 and the S8
 *                               set-up run one after another on the grid's
 *                               stream (kernel profiles without overlap);
 *                               0 (default): on their own streams.
 *   CHNS_OPT_TIME_SCHEME        CHNS_SCHEME_SPLIT (default: the first-order
 *                               split step S1..S9) or CHNS_SCHEME_CN (the
 *                               second-order Crank-Nicolson variant, two-phase
 *                               grids only; see below);
 *   CHNS_OPT_PICARD_ITERATIONS  Picard iterations per Crank-Nicolson step
 *                               (default 3).
 *   CHNS_OPT_MARCH_SWEEP_CELLS  3D multigrid levels with at least this many
 *                               cells run their smoothing and residual
 *                               sweeps marching along z with the stencil's
 *                               planes in LDS, and the CG apply of a pressure
 *                               solve on such a grid forms its face
 *                               coefficients from the cell density instead
 *                               of reading them (default 16777216: levels
 *                               whose arrays outgrow the 256 MB Infinity
 *                               Cache); >= 1.  Either form computes the same
 *                               per-cell arithmetic, bit for bit.
 *   CHNS_OPT_TILE_CYCLE_CELLS   3D multigrid levels with at most this many
 *                               cells (below the march-sweep size, above the
 *                               part solved in one workgroup) run each side
 *                               of the V-cycle as one launch over 8^3-cell
 *                               tiles that recompute their halos in LDS
 *                               instead of three grid-wide launches (default
 *                               262144: 64^3 cells and below; 0: never).
 *                               Same per-cell arithmetic, bit for bit.
 *   CHNS_OPT_TIME_GUESS         1 (default): the S7 and S8 solves of a split
 *                               step start from their solutions of the
 *                               handle's three previous steps extrapolated in
 *                               time (3 x^n - 3 x^(n-1) + x^(n-2); linear or
 *                               x^n while fewer exist), in every cell where
 *                               the incoming p^n is this handle's previous
 *                               pressure (elsewhere the history restarts);
 *                               else from the step's own guess (u^n, p^n).
 *                               0: never.  The solutions meet the same
 *                               tolerances either way (three-phase drops at
 *                               128^3: 9 -> 6 pressure and 4 -> 2 momentum
 *                               CG iterations).
 *                               chns_step_record and the adjoint's
 *                               recomputation use the step's own guesses, so
 *                               an adjoint rollout that must repeat its
 *                               forward steps bit for bit sets 0.
 * Results do not depend on CHNS_OPT_SERIAL_COMPONENTS; the two S2 solvers
 * agree to the CH tolerance.
 *
 * Crank-Nicolson variant (the paper's time scheme: every term at the
 * midpoint, v~ = (v^k + v^{k+1})/2, phi~, mu~, p~, rho(phi~), eta(phi~),
 * psi'(phi~), advection (rho~ v~ + J~/Pe) . grad v~).  The library solves
 * that nonlinear system by a fixed number of Picard iterations, each a
 * sequence of the split step's linear solves: with the previous iterate
 * phi~m, v~m, p~m,
 *   C1-C4  (I - dt/2 kM S L + dt/2 kM Cn^2 L L) phi~ = phi^k - dt/2 D(v~m A phi~m)
 *            + dt/2 kM L(psi'(phi~m) - S phi~m);  mu~ = psi'(phi~m) + S (phi~ - phi~m)
 *            - Cn^2 L phi~;  phi^{k+1} = phi^k - dt D(v~m A phi~m - kM G mu~)
 *   C5-C7  (2 rho~_f/dt) v~* - (1/Re) div(eta~ grad v~*) = (2 rho~_f/dt) v^k
 *            - (m~ . grad) v~m - (1/We) G p~m - (1/(We Cn)) A(phi~m) G mu~ + rho~_f g_hat/Fr
 *   C8-C9  -D(rho~_f^{-1} G dp) = -(2 We/dt) D v~*,  v~ = v~* - dt/(2 We) rho~_f^{-1} G dp,
 *            p~ += dp
 * and v^{k+1} = 2 v~ - v^k.  At a fixed point the stabiliser term and the
 * pressure increment vanish and the midpoint system holds.  chns_step then
 * returns mu~ in mu and the midpoint pressure in p; the momentum components
 * run one after another on the grid's stream.  The adjoint, step records
 * and the energy monitor cover the split step only.                        */
enum { CHNS_OPT_CH_SOLVER = 1, CHNS_OPT_SERIAL_COMPONENTS = 2, CHNS_OPT_TIME_SCHEME = 3,
       CHNS_OPT_PICARD_ITERATIONS = 4, CHNS_OPT_MARCH_SWEEP_CELLS = 5, CHNS_OPT_TILE_CYCLE_CELLS = 6,
       CHNS_OPT_TIME_GUESS = 7 };
enum { CHNS_CH_DIRECT = 0, CHNS_CH_PCG = 1, CHNS_CH_DIRECT_DENSE = 2 };
enum { CHNS_SCHEME_SPLIT = 0, CHNS_SCHEME_CN = 1 };
int chns_set_option(struct chns_grid *g, int option, int value);

/* Release the handle (host metadata only; device memory is the caller's). */
int chns_destroy_grid(struct chns_grid *g);

/* Static text for an error code.                                          */
const char *chns_error_string(int code);

/* Copy the calling thread's most recent error message into buf (always
 * NUL-terminated when len > 0); returns its full length.                  */
int chns_last_error(char *buf, size_t len);

#ifdef __cplusplus
}
#endif

#endif /* CHNS_H */
