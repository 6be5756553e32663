/*
 * lbfs.h -- C ABI of the MI355X (gfx950) enthalpy lattice Boltzmann flux solver (LBFS)
 * for a ferrofluid droplet freezing on a cold wall in a uniform magnetic field
 * (Zhou, Yang, Wang, Wu, Niu, arXiv 2511.10257).
 *
 * One time step (Table 1 of the paper, "computational procedure"):
 *   1. magnetic potential: the compact system that the magnetic LBFS of Sec. 3.1
 *      (Eqs. 12-18) reaches at delta_t = dx/2, i.e. Eq. 4 with face permeabilities,
 *      relaxed by `sweeps` red-black Gauss-Seidel/SOR sweeps (warm started), by
 *      `sweeps` SSP-RK3 pseudo-steps of Eq. 17 itself, or by multigrid cycles
 *      (mag_method), optionally repeated until a residual target (mag_max_iters);
 *   2. Kelvin force F_mg = (mu0 chi / 2) grad |H|^2 (Eq. 6), held over the stages;
 *   3. three stages of strong-stability-preserving third-order Runge-Kutta (Eq. 46)
 *      on W = (He, p, rho cs^2 u, rho cs^2 v, C) (Eq. 39), each stage computing the
 *      LBFS face fluxes (Eq. 44 reconstruction, Eq. 45 compatibility, star
 *      distributions Eqs. 16/22/32/33, moments Eq. 43) and the sources (Eq. 41);
 *   4. Eq. 8 (liquid fraction and temperature) after the step (Table 1 (d)) and the
 *      lagged dFs/dt of Eqs. 9-10.
 * The observables (Eq. 51 and the quantities of Figs. 11, 12 and 15) are reduced in
 * FP64 only when lbfs_observe is called, the "if output required" branch of Table 1;
 * a step writes no partial sums.
 * Lattice units: c = 1, cs^2 = 1/3, streaming step delta_t = dx/2.
 *
 * Conventions
 *  - Every function returns an int status (LBFS_OK or a negative LBFS_E_*), except
 *    lbfs_state_bytes (0 on invalid parameters), lbfs_strerror and lbfs_destroy.
 *  - The caller owns the parameter block, every host buffer and the device buffer
 *    passed to lbfs_init (it must stay allocated until lbfs_destroy). The library owns
 *    the handle. The HIP stream is borrowed; all device work is enqueued on it.
 *  - Fields are nx*ny arrays, row-major (index j*nx + i), cell (i,j) centred at
 *    ((i+1/2)dx, (j+1/2)dx). Host arrays exchanged through the ABI are FP64.
 *  - A handle is not thread safe: use one handle per host thread.
 *  - Precision is fixed at init; observables are always FP64.
 */
#ifndef LBFS_H
#define LBFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBFS_ABI_VERSION 3u

enum {
    LBFS_OK = 0,
    LBFS_E_INVAL = -1,     /* invalid argument or parameter block           */
    LBFS_E_NOMEM = -2,     /* buffer too small / batch budget exhausted     */
    LBFS_E_NONFINITE = -3, /* the last reduction saw a non-finite value     */
    LBFS_E_DEVICE = -4,    /* a HIP call failed                             */
    LBFS_E_STATE = -5,     /* call out of order (e.g. step before init)     */
    LBFS_E_ABI = -6        /* abi_version mismatch                          */
};

typedef enum { LBFS_FP32 = 0, LBFS_FP64 = 1 } lbfs_precision;

/* walls: 0 = west (x = 0), 1 = east (x = nx dx), 2 = south (y = 0), 3 = north */
enum { LBFS_TBC_ADIABATIC = 0, LBFS_TBC_FIXED = 1 };     /* thermal wall condition  */
enum { LBFS_MBC_INSULATING = 0, LBFS_MBC_FIXED = 1 };    /* magnetic wall condition:
                                                            fixed = potential of the
                                                            applied uniform field  */
enum { LBFS_INIT_DROPLET = 0, LBFS_INIT_UNIFORM = 1 };
enum { LBFS_MAG_SWEEPS = 0, LBFS_MAG_LBFS = 1, LBFS_MAG_MULTIGRID = 2 };   /* per-step magnetic update */

/* Problem statement (plain data, copied at init). Phase-indexed arrays are
   [solid, liquid, gas]; Eq. 11 mixes them with the solid fraction Fs and the
   clamped order parameter. */
typedef struct lbfs_params {
    uint32_t abi_version;     /* = LBFS_ABI_VERSION                                 */
    int32_t nx, ny;           /* cells, each 4..2^20, nx * ny <= 2^30               */
    int32_t precision;        /* lbfs_precision                                     */
    double dx;                /* cell size                                          */
    double dt;                /* Runge-Kutta time step; 0: min(dx/2, 0.4 dx^2 / D_max)
                                 with D_max the largest kinematic viscosity or thermal
                                 diffusivity of the three phases                     */
    double dt_stream;         /* streaming step delta_t; 0 or dx/2 (only dx/2 is supported) */
    double rho[3], mu[3], cp[3], lambda[3], chi[3];
    double latent;            /* latent heat L (Eq. 7)                              */
    double t_melt;            /* solidus Ts (Eq. 8); the melting point Tm of Eq. 50 */
    double t_init;            /* initial temperature                                */
    double mu0;               /* vacuum permeability (Eq. 2)                        */
    double h0;                /* applied field strength                             */
    double field_angle_deg;   /* direction of the applied field, from +x            */
    double gravity[2];        /* F_g = rho g (Eq. 9)                                */
    double sigma, xi;         /* interfacial tension, interface thickness (Sec. 2)  */
    double mobility;          /* M_c (Eq. 10)                                       */
    double tau_g;             /* phase-field relaxation parameter, > 1/2            */
    double drop_cx, drop_cy, drop_radius;   /* initial droplet (Fig. 8)             */
    int32_t init_kind;        /* LBFS_INIT_*                                        */
    double c_init;            /* order parameter of LBFS_INIT_UNIFORM               */
    int32_t periodic[2];      /* periodic x / y (then the walls of that axis are unused) */
    int32_t thermal_bc[4];    /* LBFS_TBC_* per wall                                */
    double thermal_val[4];    /* wall temperatures of fixed walls                   */
    int32_t mag_bc[4];        /* LBFS_MBC_* per wall                                */
    int32_t sweeps;           /* magnetic iterations per step: red-black sweeps, or
                                 pseudo-time steps with LBFS_MAG_LBFS                */
    double sor_omega;         /* relaxation factor of the per-step sweeps (0, 2)    */
    double init_omega;        /* SOR factor of the initial solve, <= 0: automatic   */
    double init_tol;          /* relative residual target of the initial solve      */
    int32_t init_max;         /* sweep cap of the initial solve                     */
    int32_t init_check;       /* sweeps between residual checks of the initial solve */
    /* Per-step magnetic update (the initial solve always uses the sweeps; both methods
       have the same fixed point): LBFS_MAG_SWEEPS relaxes the compact system of the
       magnetic LBFS flux (Sec. 3.1 at delta_t = dx/2) by red-black SOR; LBFS_MAG_LBFS
       advances Eq. 17 in pseudo-time by SSP-RK3, the paper's own procedure (Table 1
       (b)-(c)), with the face flux -D mu_f (phi_R - phi_L) / dx that the m* moments of
       Eqs. 13, 16 and 44 reduce to at delta_t = dx/2. Only D * dtau matters. */
    int32_t mag_method;       /* LBFS_MAG_*; LBFS_MAG_MULTIGRID (not in the paper) runs
                                 `sweeps` geometric multigrid V(2,2) cycles of the same
                                 compact system per step (walls on every side, no
                                 convergence control; the initial solve uses cycles too) */
    double mag_lbfs_d;        /* D of tau_m = 1/2 + mu D / (cs^2 delta_t), > 0 (also
                                 checked when the sweeps are the per-step method)    */
    double mag_lbfs_dtau;     /* pseudo-time step; 0: dx^2 / (4 D mu_max), mu_max =
                                 mu0 max_k (1 + chi_k), stable for every mode        */
    /* Convergence control of the per-step magnetic update (either method): with
       mag_max_iters > 0 the step repeats chunks of `sweeps` iterations until
       ||r||_2 <= mag_tol (checked on the device after each chunk) or mag_max_iters
       iterations (rounded up to whole chunks); every chunk is launched, and a converged
       instance's chunks only copy the potential, so the step stays one graph. */
    int32_t mag_max_iters;    /* 0: exactly `sweeps` iterations per step; <= 100000 */
    double mag_tol;           /* absolute target of ||r||_2 (>= 0)                  */
    /* Contact angle of each wall through the liquid, degrees in (0, 180) (Sec. 4.2
       wetting; the paper gives no condition): the order parameter's ghost cells carry
       n.grad C = -(4/xi) cos(theta) C (1 - C), n into the fluid, the gradient of the
       equilibrium profile meeting the wall at theta; 90 is the plain mirror. */
    double contact_angle_deg[4];
    double t_liquidus;        /* liquidus Tl >= t_melt (Eq. 8); Ts = Tl = Tm by default */
} lbfs_params;

typedef struct lbfs_observables {
    double t;                 /* simulated time                                     */
    double liquid_fraction;   /* sum(Ct Fl) / sum(Ct), Ct = clamp(C, 0, 1)          */
    double solid_ratio;       /* Q_L of Eq. 51: sum(Fs dA) / A0                     */
    double volume;            /* sum(Ct dA)                                         */
    double volume0;           /* A0: volume at initialisation                       */
    double mag_residual;      /* ||r||_2 of the magnetic system after the sweeps    */
    double umax;              /* max |u| over all cells                             */
    double umax_drop;         /* max |u| over cells with Ct >= 1/2                  */
    double height;            /* sum(Ct dx) along the column containing drop_cx     */
    double wall_heat;         /* sum over the south wall of -lambda dT/dy dx (fixed wall) */
    double fourier;           /* Fo of Eq. 50: lambda_l t / (rho_l Cp_l R0^2), R0 = drop_radius */
    double peclet;            /* Pe of Eq. 50 as umax_drop D / alpha_l, D = 2 R0,
                                 alpha_l = lambda_l / (rho_l Cp_l) (printed with a square
                                 that makes it dimensional; read as the usual u D / alpha) */
    /* Droplet shape from the moments of Ct (Sec. 4.3 deformation ratio b/a): centroid;
       2 sqrt of the Ct-weighted variance along x and along y; the same along the
       principal axes of the covariance, and the major axis direction (degrees from +x,
       in (-90, 90]). An ellipse of semi-axes a, b gives a and b exactly. */
    double centroid_x, centroid_y;
    double semi_axis_x, semi_axis_y;
    double semi_axis_major, semi_axis_minor, major_axis_deg;
    double solid_height;      /* sum(Fs dx) along the column containing drop_cx: the
                                 frozen part of the height (Fig. 17, freezing front)   */
    int64_t step;
    int32_t nonfinite;        /* 1 if a conserved value was not finite              */
} lbfs_observables;

/* field ids for lbfs_read_field / lbfs_write_field */
enum {
    LBFS_FIELD_HE = 0, LBFS_FIELD_P = 1, LBFS_FIELD_MX = 2, LBFS_FIELD_MY = 3,
    LBFS_FIELD_C = 4,         /* conserved: He, p, rho cs^2 u, rho cs^2 v, C        */
    LBFS_FIELD_PHI = 5,       /* magnetic potential phi_m (full, Eq. 3)             */
    LBFS_FIELD_S = 6,         /* lagged dFs/dt                                      */
    LBFS_FIELD_T = 7,         /* temperature, Eq. 8 (read only)                     */
    LBFS_FIELD_FL = 8         /* liquid fraction, Eq. 8 (read only)                 */
};

typedef struct lbfs_solver lbfs_solver;
typedef struct lbfs_batch lbfs_batch;

/* Fill p with the defaults of the synthetic freezing-droplet workload for an nx x ny
   box (property ratios of the paper's Sec. 5 table, lattice values stable for the
   explicit scheme). */
int lbfs_params_default(lbfs_params* p, int32_t nx, int32_t ny, int32_t precision);

/* Eq. 50: set latent = Cp_l (Tm - t_wall) / ste and h0 = sqrt(bo_m sigma / (mu0 D)),
   D = 2 drop_radius; also sets the south wall to the fixed temperature t_wall and the
   field direction. */
int lbfs_params_from_dimless(lbfs_params* p, double ste, double t_wall, double bo_m,
                             double angle_deg);

/* Bytes of device memory one solver needs for these parameters; 0 if invalid. */
size_t lbfs_state_bytes(const lbfs_params* p);

/* The "Initialization" block of Table 1: validate p, carve the state out of dev_buf
   (>= lbfs_state_bytes(p) bytes, caller owned; LBFS_E_NOMEM if smaller), initialise
   the fields (the half droplet on the cold wall of Fig. 8, or a uniform state: He
   from Eq. 8 inverted at t_init, fluid at rest, p = 0) and converge the magnetic
   potential of Eq. 4 for that state. stream is a hipStream_t (NULL = default stream).
   *out receives the handle (owned by the library, released by lbfs_destroy).
   LBFS_E_ABI on an abi_version mismatch, LBFS_E_INVAL on invalid parameters,
   LBFS_E_DEVICE if a HIP call fails. Synchronous. */
int lbfs_init(const lbfs_params* p, void* dev_buf, size_t bytes, void* stream,
              lbfs_solver** out);

/* Enqueue nsteps time steps on the stream (asynchronous). On a non-default stream and
   a grid of fewer than 2^19 cells the steps are replays of HIP graphs captured on first
   use: each replay covers the longest of 16, 8, 4 or 2 consecutive steps that the steps
   still to go fill, and a last single step is launched directly (LBFS_GRAPH_STEPS=k in
   the environment at init sets the longest length, 1..64, the others being the powers
   of two below it). Larger grids launch their kernels directly, where graphs gain
   nothing (LBFS_GRAPH=1 at init replays graphs there too); LBFS_NO_GRAPH=1 launches
   directly at every size. The results are the same either way. */
int lbfs_step(lbfs_solver* s, int32_t nsteps);

/* Capture and instantiate now every HIP graph that lbfs_step and lbfs_step_profiled
   replay (every length, from either potential buffer), and create the timing events of
   a profiled run that samples up to 16 steps, so that the first steps after init,
   lbfs_set_tile_shapes or lbfs_autotune pay for neither. Enqueues no work; the state
   and the clock are unchanged. Captures nothing where steps are not graph replays
   (default stream, large grids, LBFS_NO_GRAPH=1). LBFS_E_STATE on a borrowed batch handle,
   LBFS_E_DEVICE if a capture or an event creation fails. */
int lbfs_prepare(lbfs_solver* s);

/* Kernel kinds of one step, for lbfs_step_profiled: the magnetic phase (one launch
   per 4 sweeps: permeability, sweeps, residual) and the three Runge-Kutta stages
   (the third also applies Eq. 8 and stores the lagged dFs/dt). REDUCE, the FP64
   reduction of the observables (per-tile partial sums, then one sum per instance),
   runs in lbfs_observe and is not timed here. */
enum { LBFS_K_MAG = 0, LBFS_K_STAGE1, LBFS_K_STAGE2, LBFS_K_STAGE3, LBFS_K_REDUCE, LBFS_NKERNELS };

/* lbfs_step with the kernel phases of every sample_every-th step timed: their launches
   (hipExtLaunchKernelGGL on the solver's stream) record the start of the phase's first
   kernel and the end of its last into HIP events (sample_every >= 1; at most 4096
   sampled steps; the other steps run as in lbfs_step). Synchronises at the end and
   writes, per kind, the mean duration of one phase in ms (kernel_ms[LBFS_NKERNELS]) and
   the number of timed phases (launches[LBFS_NKERNELS]). */
int lbfs_step_profiled(lbfs_solver* s, int32_t nsteps, int32_t sample_every, double* kernel_ms,
                       int32_t* launches);

/* lbfs_step_profiled in two calls, so that a caller can time the steps alone with its
   own clock (start, synchronise the stream, read the clock, then collect):
   lbfs_step_profiled_start enqueues the steps and their timing events and returns at
   once (asynchronous, like lbfs_step); lbfs_profile_result waits for the stream and
   writes kernel_ms and launches as lbfs_step_profiled does. One profiled run may be
   pending per solver: LBFS_E_STATE from a start (or lbfs_step_profiled) while one is
   pending, and from a result call with none pending. */
int lbfs_step_profiled_start(lbfs_solver* s, int32_t nsteps, int32_t sample_every);
int lbfs_profile_result(lbfs_solver* s, double* kernel_ms, int32_t* launches);

/* The "if output required" branch of Table 1. Synchronise the stream, reduce the
   current state in FP64 (fixed order) and return its observables in *o (caller owned):
   the solid ratio Q_L of Eq. 51, the liquid fraction, the height and frozen height
   along the centre column (Fig. 11, Fig. 17), the wall heat (Fig. 15), max |u| and the
   Peclet and Fourier numbers of Eq. 50 (Fig. 12), and the droplet shape moments. The
   state is the one after the last step, or as last written by lbfs_write_field or
   lbfs_load_state (mag_residual is the one the last magnetic phase left). Returns
   LBFS_E_NONFINITE (with o filled) when the state holds a non-finite value,
   LBFS_E_INVAL on a NULL argument. */
int lbfs_observe(lbfs_solver* s, lbfs_observables* o);

/* One evaluation of R(W) (Eq. 46) for the current state, with the Kelvin force of the
   current potential and the stored lagged dFs/dt; host_R is 5*nx*ny FP64,
   field-major (He, p, Mx, My, C). Synchronous. */
int lbfs_rhs(lbfs_solver* s, double* host_R);

/* Run nsweeps red-black sweeps of the magnetic system with factor omega on the
   current state; *residual receives ||r||_2 afterwards. Synchronous. */
int lbfs_mag_sweeps(lbfs_solver* s, int32_t nsweeps, double omega, double* residual);

/* Advance the magnetic potential by nsteps SSP-RK3 pseudo-time steps of the LBFS
   solve (Sec. 3.1, Eq. 17) with the instance's D and dtau, whatever its per-step
   method, on the permeability of the current state; *residual receives ||r||_2
   afterwards. LBFS_E_STATE on a borrowed batch handle. Synchronous. */
int lbfs_mag_pseudo_steps(lbfs_solver* s, int32_t nsteps, double* residual);

/* Run ncycles geometric multigrid V(2,2) cycles of the compact magnetic system (the
   fixed point of the sweeps and of the LBFS pseudo-time solve; not in the paper) on the
   current state: 2 x 2 cell coarsening down to 32 cells a side, mean face weights,
   the sum of the children's residuals, the correction interpolated bilinearly, the
   coarsest level by red-black SOR in one workgroup. *residual receives ||r||_2
   afterwards. Needs walls on every side (LBFS_E_INVAL on a periodic axis);
   LBFS_E_STATE on a borrowed batch handle. Synchronous. */
int lbfs_mag_multigrid(lbfs_solver* s, int32_t ncycles, double* residual);

/* Local heat flux Q = -lambda (dT/dy) at the south wall (Sec. 5.2, Fig. 15) of the
   current state, one value per column into host_q (n = nx): the second-order one-sided
   difference through the wall temperature and the first two cell centres, lambda of
   the wall cell (Eq. 11). All zero unless the south wall holds a fixed temperature.
   Also valid on a borrowed batch handle. Synchronous. */
int lbfs_wall_heat_profile(lbfs_solver* s, double* host_q, size_t n);

/* Copy a field to / from a host FP64 array of n = nx*ny values. Synchronous. After a
   write (as after lbfs_load_state) the next magnetic phase derives the permeability
   from the written state itself; otherwise it reads the one the last step's stage 3
   left. */
int lbfs_read_field(lbfs_solver* s, int32_t field, double* host, size_t n);
int lbfs_write_field(lbfs_solver* s, int32_t field, const double* host, size_t n);

/* Set the clock (time and step count) of the solver. */
int lbfs_set_time(lbfs_solver* s, double t, int64_t step);

/* Checkpoint: raw state in the native precision plus clock; resume is bitwise. */
size_t lbfs_checkpoint_bytes(const lbfs_solver* s);
int lbfs_save_state(lbfs_solver* s, void* host, size_t bytes);
int lbfs_load_state(lbfs_solver* s, const void* host, size_t bytes);

/* ------------------------------------------------------------------ tile shapes
 * Every kernel works on a list of rectangular tiles. The stage kernels and the magnetic
 * kernel each have a small table of candidate tile shapes (cells per tile and threads
 * per workgroup); the results do not depend on the shape (each cell and face is
 * computed by the same arithmetic), only the time does. The first shape of each table
 * is the default, except above 2^17 cells for the magnetic kernel (its third shape,
 * 64 x 16, and above 512 x 512 cells its second, 64 x 32) and above 512 x 512 cells for
 * the FP64 stage kernels (their fifth shape, 12 x 7). */

#define LBFS_MAX_SHAPES 8

/* kind 0: stage kernels, 1: magnetic kernel. With index < 0 returns the number of
   shapes of that kind; otherwise writes the tile (tx x ty cells), the workgroup size
   (threads) and flags of shape `index` (bit 0: the first two stages load the owned
   cells' values before the halo rather than after the faces). Any pointer may be NULL.
   Kind 1 has one more index, equal to the count: no magnetic launch, the step's
   red-black sweeps run inside Runge-Kutta stage 1 on its tiles (a halo of
   2 MAG_KMAX + 3 = 11 cells in LDS, the same arithmetic, so the same results bit for
   bit); flags bit 1 marks it, tx = ty = threads = 0. It needs the sweeps as the
   per-step method, no convergence control and at most 4 sweeps per step. */
int lbfs_tile_shape(int32_t kind, int32_t precision, int32_t index, int32_t* tx, int32_t* ty, int32_t* threads,
                    int32_t* flags);

/* Use the given shapes from the next launch on (a changed magnetic shape recomputes the
   residual as lbfs_autotune does); mag_shape equal to the magnetic shape count selects
   the sweeps inside stage 1 (LBFS_E_INVAL where that is not possible) and keeps the
   current magnetic tiles for the initial solve and lbfs_mag_sweeps. Synchronous. */
int lbfs_set_tile_shapes(lbfs_solver* s, int32_t stage_shape, int32_t mag_shape);

/* The shapes the next launches use (indices into the tables of lbfs_tile_shape). */
int lbfs_tile_shapes_in_use(const lbfs_solver* s, int32_t* stage_shape, int32_t* mag_shape);

/* Autotuner: time whole time steps (one untimed, then reps timed, kernels launched
   directly) from this solver's current state with every stage shape (at the current
   magnetic shape), then with every magnetic shape (at the fastest stage shape), and
   keep the fastest of each: the default (the stage shape a solver of this size and
   precision starts with, magnetic shape 0) unless another is faster by more than 2 %,
   the spread of such timings. Every candidate is timed twice, in a forward
   and a backward pass over the list, and keeps the shorter time, so that a clock that
   still rises or falls favours no position in the list. Where the sweeps can run inside stage 1, that
   variant is timed too and chosen when its step beats the best step by 2 %. Before
   each candidate and at the end the state is loaded again from a host snapshot in the
   checkpoint format (lbfs_save_state), so the state, clock and results are unchanged;
   until the next step, mag_residual then reports the residual of the current
   potential with the current permeability (a step reports it with the permeability
   of the step's start). chosen[2] receives the indices (chosen[1] the count of
   magnetic shapes for the fused variant), ms[2*LBFS_MAX_SHAPES] the mean ms per step
   (stage shapes first, magnetic shapes from index LBFS_MAX_SHAPES, then the fused
   step's time minus the best magnetic shape's); either may be NULL. Synchronous. */
int lbfs_autotune(lbfs_solver* s, int32_t reps, int32_t* chosen, double* ms);

/* Release the handle (the device buffer stays the caller's). NULL is allowed; a handle
   owned by a batch (lbfs_batch_slot) is left alone. */
void lbfs_destroy(lbfs_solver* s);

/* ------------------------------------------------------------------ no allocation
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): lbfs_step without a solver or a
 * device buffer. The caller owns the state, in device memory on the current device,
 * seven nx*ny row-major arrays (row pitch nx) in the storage lbfs_init uses:
 *   fields[0..3] He, p, rho cs^2 u, rho cs^2 v   (float for LBFS_FP32, double for FP64)
 *   fields[4]    C, the order parameter           (double in both precisions)
 *   fields[5]    phi - phi0: the potential minus the applied-field potential
 *                phi0 = -h0 (x cos a + y sin a), a the field angle (float / double)
 *   fields[6]    the lagged dFs/dt                 (float / double)
 * nsteps time steps of the problem p are enqueued on `stream` (a hipStream_t of the
 * current device; asynchronous, direct launches, the arithmetic of lbfs_step, so the
 * same fields bit for bit) and the new state is left in the same arrays. The stage
 * fields, the second potential buffer, the three fields stage 1 leaves for stages 2
 * and 3, the descriptor, the tile lists and the residual partials live in the
 * library's static scratch of the current device, at most LBFS_STATIC_SCRATCH_BYTES:
 * 64 B per cell in FP32 and 112 B in FP64 plus the lists, i.e. up to about 1.3 M cells
 * in FP32 (1024 x 1024 fits) and 0.74 M in FP64. The
 * function allocates nothing. Every call on a device uses that device's one scratch:
 * calls that overlap on one device (other streams, other threads) race; calls on one
 * stream are ordered. Every value a step reads from the scratch is written earlier in
 * the same call. No observables are reduced (read them through a solver). The call
 * enqueues kernels and at most one device-to-device copy (no memset), so it can be
 * captured into a HIP graph and replayed; the first call on a device looks up the
 * scratch's address, so make one call (nsteps = 0 will do) before a capture.
 * LBFS_E_INVAL on invalid parameters, a NULL field, nsteps < 0, multigrid or
 * convergence control (mag_max_iters > 0); LBFS_E_NOMEM if the problem does not fit
 * the scratch; LBFS_E_DEVICE if a HIP call fails. */
#define LBFS_STATIC_SCRATCH_BYTES ((size_t)80 << 20)
int lbfs_step_fields(const lbfs_params* p, void* const fields[7], int32_t nsteps, void* stream);

/* ------------------------------------------------------------------ batches
 * Many independent problems (different sizes, fields, Stefan and magnetic Bond numbers)
 * advanced together: every kernel of a step runs once over the concatenated tiles of
 * all live instances, so each instance computes exactly what it computes alone (the
 * same fields, bit for bit) while the launches fill the GPU. Instances are admitted
 * and retired between steps; their state is carved from one caller-owned device
 * buffer by a first-fit allocator (no device allocation inside the library). All
 * instances of a batch share the precision and the per-step magnetic sweeps.
 * The batch's metadata (descriptors, tile lists, FP64 results) is carved from the same
 * buffer and grows on admission. A batch handle is not thread safe. */

/* Device bytes one admission takes from the batch buffer for these parameters (its
   state; the shared metadata, descriptors and tile lists, grows with the instances'
   tile counts, by about half a byte per cell); 0 if invalid. */
size_t lbfs_batch_instance_bytes(const lbfs_params* p);

/* Create an empty batch of at most max_slots instances over dev_buf (bytes, caller
   owned, alive until lbfs_batch_destroy). precision, sweeps and sor_omega are those
   every admitted instance must have. stream as in lbfs_init. */
int lbfs_batch_create(int32_t max_slots, int32_t precision, int32_t sweeps, double sor_omega, void* dev_buf,
                      size_t bytes, void* stream, lbfs_batch** out);

/* Admit one problem: validate, carve its state, initialise it as lbfs_init does
   (synchronous). *slot_out receives its slot. LBFS_E_NOMEM when no slot is free or the
   buffer has no room for it (the batch is unchanged); LBFS_E_INVAL when p does not
   share the batch's precision, sweeps or sor_omega, or asks for LBFS_MAG_LBFS or
   convergence control (batches run a fixed number of sweeps). */
int lbfs_batch_admit(lbfs_batch* b, const lbfs_params* p, int32_t* slot_out);

/* Retire the instance in a slot (after the work already enqueued); its memory and slot
   become free. */
int lbfs_batch_retire(lbfs_batch* b, int32_t slot);

/* Enqueue nsteps time steps of every live instance (asynchronous; HIP graph replays
   of 16, 8, 4 or 2 steps and a last single step launched directly, as in lbfs_step on
   a non-default stream, recaptured after admissions and retirements). */
int lbfs_batch_step(lbfs_batch* b, int32_t nsteps);

/* lbfs_prepare for a batch: rebuilds the launch lists after admissions and retirements
   and captures the step graphs of the live instances (recaptured after the next
   admission or retirement). */
int lbfs_batch_prepare(lbfs_batch* b);

/* lbfs_step_profiled for a batch: mean duration of each kernel phase over all live
   instances. */
int lbfs_batch_step_profiled(lbfs_batch* b, int32_t nsteps, int32_t sample_every, double* kernel_ms,
                             int32_t* launches);
/* lbfs_step_profiled_start and lbfs_profile_result for a batch. */
int lbfs_batch_step_profiled_start(lbfs_batch* b, int32_t nsteps, int32_t sample_every);
int lbfs_batch_profile_result(lbfs_batch* b, double* kernel_ms, int32_t* launches);

/* Synchronise and fill out[max_slots] and live[max_slots] (1 for an occupied slot;
   out[k] is zeroed for a free slot). One reduction launch covers all instances.
   Returns LBFS_E_NONFINITE (outputs filled) if any live instance is non-finite. */
int lbfs_batch_observe(lbfs_batch* b, lbfs_observables* out, uint8_t* live);

/* Borrow the handle of a live slot for lbfs_read_field, lbfs_write_field, lbfs_rhs,
   lbfs_observe, lbfs_save_state and lbfs_load_state. lbfs_step, lbfs_step_profiled,
   lbfs_mag_sweeps and lbfs_mag_pseudo_steps on it return LBFS_E_STATE; it is valid
   until the slot is retired. */
int lbfs_batch_slot(lbfs_batch* b, int32_t slot, lbfs_solver** out);

/* lbfs_set_tile_shapes and lbfs_autotune for a batch: one shape pair for all live
   instances (and those admitted later), timed on whole steps of every live instance
   (the sweeps inside stage 1 are not a batch candidate). Until shapes are given by one
   of them, a batch takes, after every admission and retirement, the stage and magnetic
   shapes a single solve of its total cells and precision would take. */
int lbfs_batch_set_tile_shapes(lbfs_batch* b, int32_t stage_shape, int32_t mag_shape);
int lbfs_batch_autotune(lbfs_batch* b, int32_t reps, int32_t* chosen, double* ms);
int lbfs_batch_tile_shapes_in_use(const lbfs_batch* b, int32_t* stage_shape, int32_t* mag_shape);

/* Live instances, cells they hold and free bytes of the buffer (largest free block). */
int lbfs_batch_info(lbfs_batch* b, int32_t* live, int64_t* cells, size_t* largest_free);

/* Retire everything and release the handle. NULL is allowed. */
void lbfs_batch_destroy(lbfs_batch* b);

/* Static description of a status code. */
const char* lbfs_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif
