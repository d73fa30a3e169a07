/*
 * meso.h -- C ABI of the MI355X two-fluid shock/bubble solver.
 *
 * The solver advances the two-phase Euler system of Eq. (1) (Sec. 2.1:
 * partial densities z1 rho1 and z2 rho2, momentum, total energy, and the
 * non-conservative advection of the air volume fraction z1) with the
 * pressure-equilibrium closure of Sec. 2.1, stiffened-gas phases (the
 * Mie-Grueneisen form of Eq. (2) with constant reference terms, Sec. 2.2;
 * air as an ideal gas, Table 2) or a Cochran-Chan liquid (Eqs. (2)-(4),
 * Table 1).  The scheme is that of Sec. 3:
 * MUSCL-Hancock reconstruction with a van Leer (or minmod) slope limiter, HLLC
 * fluxes, dimensionally split sweeps, a CFL time step, and the pointwise stage
 * of the Strang split (z1 kept in [eps, 1 - eps]; for a reactive liquid also
 * the single-step Arrhenius reaction of Eq. (6) at the liquid temperature of
 * Eq. (5), with the reactant mass z2 rho2 lambda of Eq. (1) as a seventh
 * conserved component).
 *
 * The calls follow the paper's statement of the problem (Sec. 2.4 and Sec. 3):
 * a rectangular uniform grid with two materials, initial fields set once,
 * the state kept resident on the device and advanced to a final time, with
 * field output on request (host/device transfers only at initialisation and
 * output).
 *
 * Conventions for every call:
 *  - All functions return an mf_status (0 = success, negative = error) and
 *    never throw or abort.  A NULL solver/server handle gives
 *    MF_E_INVALID_ARG.
 *  - Host buffers are owned by the caller and only accessed during the call.
 *  - Field arrays are planes of nx*ny doubles, row-major with x fastest
 *    (index j*nx + i).  Primitive sets are 6 consecutive planes
 *    (z1, rho1, rho2, u, v, p); conserved sets are 6 consecutive planes
 *    (z1 rho1, z2 rho2, rho u, rho v, rho E, z1).  A reactive solver (liquid
 *    material with reactive = 1) has a seventh plane in both: the reaction
 *    progress lambda (primitive; the liquid's unreacted mass fraction, 1 =
 *    fresh) and the reactant mass z2 rho2 lambda (conserved).
 *  - Stepping calls only enqueue work on the solver's stream and return;
 *    errors found on the device (non-finite state, rho <= 0, rho c^2 <= 0;
 *    a given time step above the CFL bound) are latched and reported by the
 *    next synchronising call (mf_sync, mf_read_*, mf_get_time,
 *    mf_run_to_time, the diagnostics) as MF_E_NONFINITE_STATE or
 *    MF_E_CFL_VIOLATION.  After such an error the state is unspecified;
 *    the solver may be re-set (mf_set_*) or destroyed.
 *  - One solver is used from one host thread at a time.
 */
#ifndef MESO_H
#define MESO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define MF_OK                 0
#define MF_E_INVALID_ARG     -1   /* bad argument; nothing was changed      */
#define MF_E_OUT_OF_MEMORY   -2   /* device allocation or workspace too small */
#define MF_E_NONFINITE_STATE -3   /* NaN/Inf, rho <= 0 or rho c^2 <= 0 found */
#define MF_E_CFL_VIOLATION   -4   /* a given dt exceeded cfl / s_max          */
#define MF_E_DEVICE          -5   /* HIP runtime error (launch, copy, sync)  */
#define MF_E_NOT_READY       -6   /* result asked for before it exists       */
#define MF_E_BUSY            -7   /* server has no free slot or budget       */

/* Precision modes: arithmetic of the flux path / storage of the state. */
#define MF_FP64          0  /* FP64 everywhere; equals the FP64 contract bit for bit */
#define MF_FP32_FP64ACC  1  /* FP64 state, pressure inversion and update;
                               FP32 reconstruction, predictor and HLLC         */
#define MF_FP32          2  /* FP32 state and arithmetic                       */
#define MF_FP64_FAST     3  /* FP64 state and arithmetic with fused multiply-adds;
                               divisions and square roots from the hardware
                               reciprocal / reciprocal-square-root seeds refined
                               by a second-order series in their residual
                               (about one ulp each): within 1e-12
                               relative L1 of the FP64 contract per field after
                               the fixed step counts, not bit for bit          */

/* Boundary conditions (Sec. 2.4, Fig. 1): transmissive = zero-order
 * extrapolation of the edge cell; periodic = wrap (must be set on both
 * sides of an axis). */
#define MF_BC_TRANSMISSIVE 0
#define MF_BC_PERIODIC     1

/* Slope limiters (Sec. 3). */
#define MF_LIM_VANLEER 0
#define MF_LIM_MINMOD  1

/* Fields for mf_read_field. 0-5: conserved, 6-10: derived. */
#define MF_Z1RHO1 0
#define MF_Z2RHO2 1
#define MF_RHOU   2
#define MF_RHOV   3
#define MF_RHOE   4
#define MF_Z1     5
#define MF_RHO    6
#define MF_U      7
#define MF_V      8
#define MF_P      9
#define MF_C     10
/* Reactive solvers only: the seventh conserved plane, the reaction progress
 * lambda, the liquid temperature of Eq. (5) (K) and the volumetric
 * heat-release rate -z2 rho2 K Q of Sec. 4.5 (GW/m^3, 0 where there is no
 * reactant or T <= 0). */
#define MF_Z2RHO2LAM 11
#define MF_LAMBDA    12
#define MF_T2        13
#define MF_QDOT      14

/* Equation of state of a phase, in the Mie-Grueneisen form of Eq. (2),
 * p = p_ref(rho) + rho Gamma (e - e_ref(rho)):
 *  MF_EOS_STIFFENED:    p = (gamma - 1) rho e - gamma p_inf (constant reference
 *                       terms; air: the ideal gas, p_inf = 0);
 *  MF_EOS_COCHRAN_CHAN: Gamma = gamma0, p_ref and e_ref of Eqs. (3)-(4) with
 *                       the constants A, B (Pa), C, D and rho0 (Table 1).
 *  Phase 1 (the gas) must be MF_EOS_STIFFENED.
 * reactive = 1 (phase 2 only, MF_EOS_COCHRAN_CHAN only) makes the liquid an
 * explosive: single-step Arrhenius kinetics d lambda/dt = -lambda C exp(-Ta/T)
 * (Eq. (6); C = arr_C in 1/s, Ta = arr_Ta in K, Table 3) releasing heat_Q
 * J/kg (Table 3) into rho E, at the liquid temperature
 * T = (p - p_ref(rho2)) / (rho2 gamma0 cv) of Eq. (5) (cv in J/(kg K),
 * Table 1; reference temperature 0 K).  Unused members are ignored. */
#define MF_EOS_STIFFENED     0
#define MF_EOS_COCHRAN_CHAN  1

typedef struct {
    int32_t kind;
    int32_t reactive;
    double gamma;
    double p_inf;
    double gamma0, A, B, C, D, rho0;
    double cv, arr_C, arr_Ta, heat_Q;
} mf_material;

/* Uniform Cartesian grid (Sec. 3), cell sizes in metres.  1 <= nx, ny <= 2^30
 * and nx * ny <= 2^40; a boundary pair (lo, hi) is periodic on both sides or
 * on neither. */
typedef struct {
    int32_t nx, ny;
    double dx, dy;
    int32_t bc_xlo, bc_xhi, bc_ylo, bc_yhi;
} mf_grid;

/* Scheme options.  cfl in (0, 1]; z_floor in [0, 0.5) is the eps of the
 * pointwise stage; limiter MF_LIM_*; precision MF_FP*; fused = 1 runs the
 * two split sweeps of a step in one kernel (one read and one write of the
 * state), 0 runs one kernel per sweep (for cross-checking). */
typedef struct {
    double cfl;
    double z_floor;
    int32_t limiter;
    int32_t precision;
    int32_t fused;
    int32_t reserved;
} mf_options;

typedef struct mf_solver mf_solver;

/* Device bytes a solver of this grid, materials and precision needs (two
 * state copies of 6 planes -- 7 if the liquid is reactive -- plus a 256-byte
 * control block).  mat may be NULL (an inert pair).  0 for an invalid grid,
 * precision or material pair. */
size_t mf_workspace_bytes(const mf_grid *grid, const mf_material mat[2], int32_t precision);

/* Create a solver on the current HIP device.
 *  mat[0] = phase 1 (gas, the cavity content), mat[1] = phase 2 (liquid).
 *  dev_workspace: device memory of at least mf_workspace_bytes() bytes,
 *    256-byte aligned, owned by the caller and kept alive until
 *    mf_destroy; or NULL, then the library allocates and frees it.
 *  hip_stream: hipStream_t the solver enqueues all work on (NULL = the null
 *    stream); owned by the caller, must outlive the solver.
 * Errors: MF_E_INVALID_ARG (bad grid/material/option, workspace too small or
 * misaligned), MF_E_OUT_OF_MEMORY, MF_E_DEVICE.  The state is zero until set. */
int32_t mf_create(const mf_grid *grid, const mf_material mat[2], const mf_options *opt,
                  void *dev_workspace, size_t ws_bytes, void *hip_stream, mf_solver **out);

/* Set the state from host primitive planes (z1, rho1, rho2, u, v, p), 6*nx*ny
 * doubles (7*nx*ny with lambda last for a reactive solver), converted to
 * conserved variables on the device by the closure of Sec. 2.1.  Resets the latched error and computes the first time step's CFL
 * bound.  Synchronises the stream.  Time and step count are unchanged. */
int32_t mf_set_primitive(mf_solver *s, const double *prim);

/* Set the state from host conserved planes (6*nx*ny doubles, 7*nx*ny for a
 * reactive solver); in MF_FP32 mode
 * the values are rounded to float.  Same side effects as mf_set_primitive. */
int32_t mf_set_conserved(mf_solver *s, const double *cons);

/* Set the time and the step counter (its parity selects the sweep order:
 * x then y on even steps, y then x on odd steps).  Synchronises. */
int32_t mf_set_time(mf_solver *s, double t, int64_t step);

/* Enqueue one step.  dt <= 0: dt = CFL / max signal speed of the current
 * state (computed on the device; no host round trip).  dt > 0: use this time
 * step, which must not exceed that bound (the solver's cfl over the signal
 * speed bound s_max = max over cells of max((|u| + c)/dx, (|v| + c)/dy));
 * a larger dt is not taken: the step and every later one are skipped and the
 * next synchronising call reports MF_E_CFL_VIOLATION (found on the device, so
 * this call still returns MF_OK).  Does not synchronise. */
int32_t mf_step(mf_solver *s, double dt);

/* Enqueue nsteps CFL steps (nsteps >= 0).  Does not synchronise. */
int32_t mf_run_steps(mf_solver *s, int64_t nsteps);

/* Advance with CFL steps until t == t_end (the last step is shortened to land
 * on t_end exactly) or max_steps steps were taken.  Polls the device time
 * every few steps; synchronises before returning.  *steps_taken (may be NULL)
 * receives the number of steps taken by this call. */
int32_t mf_run_to_time(mf_solver *s, double t_end, int64_t max_steps, int64_t *steps_taken);

/* Wait for all enqueued work; MF_E_NONFINITE_STATE if an error was latched. */
int32_t mf_sync(mf_solver *s);

/* Copy one field (MF_* field id) as nx*ny doubles to host_out (count must be
 * nx*ny).  Derived fields use the closure of Sec. 2.1.  Synchronises. */
int32_t mf_read_field(mf_solver *s, int32_t field, double *host_out, size_t count);

/* Copy the conserved planes (6*nx*ny doubles, 7*nx*ny for a reactive solver)
 * to host_out; count must be that size.  Synchronises. */
int32_t mf_read_conserved(mf_solver *s, double *host_out, size_t count);

/* Time, completed step count and the last time step.  Synchronises. */
int32_t mf_get_time(mf_solver *s, double *t, int64_t *step, double *last_dt);

/* Diagnostics of the current state (synchronise; the closure is evaluated in
 * FP64 on the stored values; sums run in a fixed order, so results do not
 * depend on the launch geometry).
 *
 * Transverse averages of Sec. 4.2, one value per column (nx each):
 *   p_bar = (1/W) int p dy,  rho_bar = (1/W) int rho dy,
 *   u_bar = (1/(W rho_bar)) int rho u dy (density-weighted). */
int32_t mf_y_averages(mf_solver *s, double *p_bar, double *rho_bar, double *u_bar, size_t nx);

/* Domain integrals over the grid (cell area dx*dy), count must be 6 (7 for a
 * reactive solver): z1 rho1, z2 rho2, rho u, rho v, rho E, the gas volume z1
 * and the remaining reactant mass M_2,r of Eq. (10). */
int32_t mf_integrals(mf_solver *s, double *out, size_t count);

/* For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc / hipFree between steps): mf_integrals
 * with the same arguments, results and errors, but its device scratch (the
 * column sums and the integrals) is a fixed 4 MiB array in the library's
 * device memory instead of a temporary allocation, so the call allocates
 * nothing.  Limit: (3 + planes) * nx + planes <= 524288 doubles, i.e.
 * nx <= 52428 with 7 planes (58253 with 6); a wider grid gives
 * MF_E_INVALID_ARG.  Every call on one device shares that device's array:
 * calls that overlap on one device (solvers driven from several host
 * threads) race and must be serialised by the caller.  Synchronises the
 * solver's stream. */
int32_t mf_integrals_noalloc(mf_solver *s, double *out, size_t count);

/* Mass-weighted probability density on log-spaced bins (Sec. 4.5): bin k
 * covers 10^(lo + k dn) <= v < 10^(lo + (k+1) dn) of the field v (MF_P,
 * MF_RHO, or MF_QDOT of a reactive solver), collects the liquid mass
 * z2 rho2 dx dy of its cells, and
 * f_out[k] = m_k / (m_ref dn).  1 <= nbins <= 1024, dn > 0, m_ref > 0. */
int32_t mf_log_histogram(mf_solver *s, int32_t field, double lo, double dn, int32_t nbins,
                         double m_ref, double *f_out);

/* Fused transverse averages (Sec. 4.2), for x-t diagrams at every step: while
 * recording, each step also sums, per column, the pressure (FP64 closure of
 * the stored values), the density and the x momentum of the state it stores
 * -- in its store epilogue, so the state is not read a second time -- and
 * writes one row of 3*nx doubles (p_bar, rho_bar, u_bar as in mf_y_averages)
 * to dev_rows: row r (dev_rows + 3*nx*r) is the state after the r-th step
 * enqueued since this call, or NaN for a step the device skipped (an error,
 * or run-to-time at its end).  dev_rows: device memory of at least
 * 3*nx*max_rows doubles, owned by the caller and kept alive while recording.
 * After max_rows rows, steps are taken without recording; dev_rows = NULL
 * stops recording.  Each column is summed segment by segment (the rows of a
 * segment of the launch in increasing j, then the segments in increasing j),
 * so a value may differ from mf_y_averages of the same state by up to 2 ny u
 * of the sum of magnitudes (u = 2^-53), and depends on nothing but the grid
 * and the launch geometry.  Fused solvers (mf_options.fused = 1) only; the
 * first call allocates 3*nx*(segments) doubles of partial sums, freed by
 * mf_destroy.  MF_E_INVALID_ARG (unfused solver, max_rows < 1, misaligned
 * pointer), MF_E_OUT_OF_MEMORY.  Enqueues nothing itself. */
int32_t mf_record_averages(mf_solver *s, double *dev_rows, int64_t max_rows);

/* Rows enqueued since recording started (complete once the stream has run
 * them, e.g. after mf_sync).  Does not synchronise. */
int32_t mf_recorded_rows(mf_solver *s, int64_t *rows);

/* Fused domain integrals, for the remaining reactant mass M_2,r(t) of Eq.
 * (10) and the global rate of Eq. (11) at every step: while recording, each
 * step also sums every conserved plane of the state it stores, in its store
 * epilogue, and writes one row of nc + 1 doubles to dev_rows -- the values of
 * mf_integrals (z1 rho1, z2 rho2, rho u, rho v, rho E, z1 and, reactive,
 * M_2,r; nc = 6 or 7), then the time of that state, so that the rate of Eq.
 * (11) is the difference of consecutive rows: row r is the state after the
 * r-th step enqueued since this call, all NaN for a step the device skipped.  Each workgroup sums its cells
 * (a column's rows in order, then a fixed tree over its columns) and the
 * workgroup sums are added in launch order, so a value may differ from
 * mf_integrals of the same state by up to 2 N u of the sum of magnitudes
 * (N cells, u = 2^-53) and depends on nothing but the grid and the launch
 * geometry.  dev_rows: device memory of at least (nc+1)*max_rows doubles, owned
 * by the caller and kept alive while recording; NULL stops.  Fused solvers
 * only; the first call allocates nc doubles per workgroup of the step launch
 * (freed by mf_destroy).  MF_E_INVALID_ARG (unfused solver, max_rows < 1,
 * misaligned pointer), MF_E_OUT_OF_MEMORY.  Enqueues nothing itself. */
int32_t mf_record_integrals(mf_solver *s, double *dev_rows, int64_t max_rows);

/* Fused mass-weighted PDF (Sec. 4.5) at every step: while recording, each
 * step also adds the liquid mass z2 rho2 dx dy of every cell it stores to the
 * log-spaced bin of its field value, in its store epilogue, with the bins,
 * field and arguments of mf_log_histogram (MF_P, MF_RHO or, reactive,
 * MF_QDOT; bin edges 10^(lo + k dn); f = m_k / (m_ref dn)), and writes one row
 * of nbins doubles to dev_rows: row r after the r-th step enqueued since this
 * call, NaN for a step the device skipped.  The bins collect in the
 * workgroup's local memory, then one atomic addition per workgroup and
 * non-empty bin: a bin may differ from mf_log_histogram of the same state by
 * the order of its additions (up to 2 N u of the bin's mass); a cell whose
 * value lies within rounding of a bin edge may fall in the neighbouring bin
 * (the recording kernels of the fast modes fuse multiply-adds in the FP64
 * closure).  dev_rows: device memory of at least nbins*max_rows doubles,
 * owned by the caller; NULL stops.  Fused solvers only.  The bin edges are
 * copied to library-owned device memory (1025 doubles, allocated on first
 * use): synchronises the solver's stream.  MF_E_INVALID_ARG (as for
 * mf_log_histogram, or an unfused solver, max_rows < 1, misaligned pointer),
 * MF_E_OUT_OF_MEMORY, MF_E_DEVICE. */
int32_t mf_record_histogram(mf_solver *s, int32_t field, double lo, double dn, int32_t nbins,
                            double m_ref, double *dev_rows, int64_t max_rows);

/* Rows enqueued by the three fused records since each was started: counts[0]
 * averages, counts[1] integrals, counts[2] histogram.  Does not
 * synchronise. */
int32_t mf_recorded_counts(mf_solver *s, int64_t counts[3]);

/* Kernel timing: when enabled, every step kernel launch is bracketed by HIP
 * events on the solver's stream.  mf_kernel_time synchronises and returns the
 * summed duration (ms) and launch count of the state-update kernels since
 * the last reset (enable resets).  Costs two event records per launch. */
int32_t mf_enable_timing(mf_solver *s, int32_t enable);
int32_t mf_kernel_time(mf_solver *s, double *total_ms, int64_t *launches);

/* Measurement reference: copy `bytes` bytes from src to dst (device
 * pointers, 16-byte aligned, not overlapping; owned by the caller) with a
 * plain HIP kernel on hip_stream (NULL = the null stream), one read and one
 * write per byte like the algorithmic traffic of a step.  variant 0-3: 1 or 4
 * 16-byte vectors per thread per trip (bit 0), ordinary or non-temporal
 * loads and stores (bit 1); workgroups: grid size (0 = 8 per compute unit).
 * Enqueues only.  MF_E_INVALID_ARG for NULL or misaligned pointers or a bad
 * variant, MF_E_DEVICE if the launch fails. */
int32_t mf_stream_copy(const void *src, void *dst, size_t bytes, int32_t variant,
                       int32_t workgroups, void *hip_stream);

/* Kernel launch geometry of the state-update kernel for this solver:
 * workgroups, threads per workgroup, and the number of cells one leading
 * workgroup writes (strip width x segment height).  The segment height is
 * chosen at creation from the grid, the precision mode and the device's
 * compute units (short segments for small grids, so that every compute unit
 * gets several workgroups; on large grids taller segments down to a tail of
 * shorter ones, dispatched last, which evens out the end of the launch).  The
 * environment variable MESO_SEG_H (>= 1) fixes a uniform height, and
 * MESO_SEG_TAPER = "h2,rows" gives the last `rows` or more rows segments of h2
 * rows (h2 below the leading height; "0,0": none).  No result depends on
 * either. */
int32_t mf_launch_info(mf_solver *s, int64_t *workgroups, int32_t *threads, int32_t *tile_w,
                       int32_t *tile_h);

/* ------------------------------------------------------------------------
 * Continuous-batching server: many independent solves of different grid
 * sizes share one device.  Each admitted solve holds a slot and a block of a
 * fixed device arena (its state copies, control block and a read-back area);
 * every tick advances all admitted solves by one CFL step with one batched
 * state-update launch per class of liquid (stiffened gas, inert and reactive
 * Cochran-Chan) over a table of (solve, strip, segment) tiles.  The rows per
 * segment follow the load: few solves get short segments (more workgroups in
 * flight), a full device taller ones (less halo work), and then each solve's
 * last rows go into quarter-height segments dispatched after all the others;
 * the environment variable MESO_SERVE_SEG_H (>= 1) fixes a uniform height,
 * MESO_SERVE_TAPER = "h2,rows" the tail ("0,0": none).  Solves
 * that finish are read back on a second stream while the others keep running;
 * their slot and memory are then reused by queued requests (first come, first
 * served).  Each solve's arithmetic is exactly that of a lone mf_solver with
 * the same options, so its result does not depend on what it shares the
 * device with.
 * ------------------------------------------------------------------------ */

typedef struct mf_server mf_server;

/* hbm_budget: bytes of device memory the server may hold for solves (one
 *   arena allocated at creation); max_slots: most solves on the device at
 *   once; precision and limiter: shared by all requests; max_inflight: ticks
 *   enqueued ahead of the device before mf_server_tick waits (>= 1). */
typedef struct {
    size_t hbm_budget;
    int32_t max_slots;
    int32_t precision;
    int32_t limiter;
    int32_t max_inflight;
} mf_server_config;

/* Request states reported by mf_server_poll. */
#define MF_REQ_QUEUED  0
#define MF_REQ_RUNNING 1
#define MF_REQ_DONE    2
#define MF_REQ_FAILED  3

/* Aggregate counters of a server. */
typedef struct {
    int64_t ticks;            /* batched steps launched                      */
    int64_t cell_updates;     /* sum over ticks of the cells advanced        */
    int64_t completed;        /* requests finished (done or failed)          */
    int64_t peak_bytes;       /* largest arena use so far                    */
    int64_t bytes_in_use;     /* arena use now                               */
    int32_t active;           /* solves advancing                            */
    int32_t queued;           /* requests waiting for admission              */
    int32_t draining;         /* finished solves being read back             */
    int32_t reserved;
} mf_server_stats;

/* Device bytes one request of this grid and these materials (NULL: an inert
 * pair) needs inside the arena; 0 for an invalid grid, precision or pair. */
size_t mf_server_request_bytes(const mf_grid *grid, const mf_material mat[2], int32_t precision);

/* Create a server on the current device.  hip_stream: stream for the batched
 * steps (NULL: the server creates its own non-blocking stream); the read-back
 * stream is always the server's own.  Errors: MF_E_INVALID_ARG,
 * MF_E_OUT_OF_MEMORY (arena allocation), MF_E_DEVICE. */
int32_t mf_server_create(const mf_server_config *cfg, void *hip_stream, mf_server **out);

/* Queue one solve: grid, materials (gas, liquid; the liquid may be reactive),
 * options (cfl, z_floor; limiter and precision must equal the server's; fused
 * is ignored), host primitive planes (6*nx*ny doubles, 7*nx*ny with lambda
 * last for a reactive liquid; copied during the call) and the number of CFL
 * steps to take (>= 1).  *ticket receives the request id.  MF_E_OUT_OF_MEMORY
 * if the request can never fit in the budget. */
int32_t mf_server_submit(mf_server *srv, const mf_grid *grid, const mf_material mat[2],
                         const mf_options *opt, const double *prim, int64_t nsteps,
                         uint64_t *ticket);

/* One scheduling round: collect finished read-backs, admit queued requests
 * while a slot and arena memory are free, and enqueue one batched step of all
 * admitted solves.  Waits only when max_inflight ticks are already queued on
 * the device.  *active / *queued (may be NULL) receive the counts after it. */
int32_t mf_server_tick(mf_server *srv, int32_t *active, int32_t *queued);

/* State of a request (MF_REQ_*); MF_E_INVALID_ARG for an unknown ticket. */
int32_t mf_server_poll(mf_server *srv, uint64_t ticket, int32_t *state);

/* Tickets of requests that reached MF_REQ_DONE or MF_REQ_FAILED since they were
 * last reported here, oldest first: up to `capacity` of them are written to
 * tickets[] (host array owned by the caller) and their number to *count; the
 * rest are kept for the next call.  Each ticket is reported once.  Lets a
 * serving loop find finished work without polling every outstanding ticket. */
int32_t mf_server_finished(mf_server *srv, uint64_t *tickets, int32_t capacity, int32_t *count);

/* Copy a finished request's conserved planes (6*nx*ny doubles, 7*nx*ny for a
 * reactive liquid; count must be that size), its final time and step count,
 * and forget the request.  MF_E_NOT_READY while it runs,
 * MF_E_NONFINITE_STATE if its state became non-physical (the ticket is then
 * released as well).  Until its result is taken, a finished request holds a
 * pinned host buffer of its size. */
int32_t mf_server_result(mf_server *srv, uint64_t ticket, double *out_cons, size_t count,
                         double *t, int64_t *steps);

/* Tick until every submitted request is finished and read back. */
int32_t mf_server_drain(mf_server *srv);

int32_t mf_server_get_stats(mf_server *srv, mf_server_stats *st);

/* Wait for the device, release every resource; pending tickets are lost. */
int32_t mf_server_destroy(mf_server *srv);

/* Release the solver (and the workspace if the library allocated it).
 * Synchronises its stream first. */
int32_t mf_destroy(mf_solver *s);

/* Static text for a status code. */
const char *mf_status_str(int32_t status);

/* Library version string. */
const char *mf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MESO_H */
