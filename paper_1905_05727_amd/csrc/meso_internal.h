// meso_internal.h -- device-side layout shared by the HIP kernels and the
// host side of the C ABI (not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "meso.h"

namespace meso {

// Step kernel geometry: one workgroup = one wave64 x 4 = 256 threads, thread t
// owns column x0 - 2 + t of a strip; the two columns on each side are the
// stencil halo of a sweep, so a strip writes 252 columns.
constexpr int kThreads = 256;
constexpr int kHalo = 2;
constexpr int kTileW = kThreads - 2 * kHalo;
// Largest y dimension of a launch grid: the segments of one strip.
constexpr int kMaxSegs = 65535;

// Precision modes (same numbering as MF_FP64 / MF_FP32_FP64ACC / MF_FP32 /
// MF_FP64_FAST).
enum { kP64 = 0, kPMix = 1, kP32 = 2, kP64F = 3 };
// Step kernel variants: fused x-then-y, fused y-then-x, single x sweep,
// single y sweep.
enum { kXY = 0, kYX = 1, kX = 2, kY = 3 };

// Device control block of one solve: time, step counter, the CFL maximum of
// the state (two slots, alternating with the step parity), latched errors.
struct alignas(256) Control {
    double t;
    double dt;
    double lam_x, lam_y;     // dt/dx, dt/dy of the step being executed
    double hl_x, hl_y;       // 0.5 * lam
    unsigned long long smax_bits[2];  // bit pattern of the max signal speed / h
    long long step;          // completed steps
    long long step_exec;     // index of the step being executed
    int skip;                // 1: the enqueued step does nothing
    int err;                 // latched error bits (1 = bad state, 2 = dt above the CFL bound)
};

// Everything a step kernel needs to know about one solve.
struct Desc {
    void *buf[2];            // two state copies, nc planes each
    Control *ctl;
    int nx, ny;
    int pitch;               // elements per row
    int seg_h;               // rows per workgroup segment
    long long plane;         // elements per plane
    int bc_xlo, bc_xhi, bc_ylo, bc_yhi;
    int nstrips, nsegs;
    // segments 0 .. seg_n1-1 are seg_h rows tall, the rest (from row
    // seg_n1 * seg_h on, dispatched last) seg_h2 rows: a tail of short
    // segments evens out the end of a launch
    int seg_n1, seg_h2;
    double dx, dy, cfl;      // cell sizes and CFL number (used by the batched dt kernel)
    double idx, idy;         // 1/dx, 1/dy
    double zlo, zhi;         // eps, 1 - eps of the pointwise stage
    double g1, g2, h1, h2;   // mixture constants 1/Gamma_k, phi_k of stiffened gases
    int eos2;                // liquid EoS: 0 stiffened gas, 1 Cochran-Chan
    int nc;                  // conserved planes: 6, or 7 with the reactant mass
    // Cochran-Chan liquid: A, B, C, D, rho0, 1/Gamma0, -A/(rho0(1-C)), B/(rho0(1-D)),
    // A*C, B*D
    double cA, cB, cC, cD, crho0, ciG, ckA, ckB, cAC, cBD;
    // reactive liquid: Gamma0 and c_v (temperature, Eq. (5)); Arrhenius C, Ta
    // and heat of reaction Q (Eq. (6), Table 3)
    double cG0, rxcv, rxC, rxTa, rxQ;
    // A recording step (diagnostics summed in the store epilogue); each
    // pointer is nullptr when that quantity is not recorded.
    //  diag: per segment s, 3 * nx column sums of pressure, density and x
    //        momentum at diag + 3 * nx * s (transverse averages);
    //  dint: per workgroup (strip bx, segment by), the sums of the nc stored
    //        planes at dint + nc * (by * nstrips + bx) (domain integrals);
    //  dhist: the liquid mass z2 rho2 dx dy of the stored cells per bin of
    //        field hfield (MF_P, MF_RHO or MF_QDOT) over the hbins + 1
    //        ascending edges hedges, accumulated into dhist (zeroed before
    //        the step).
    //  hlo, hidn: lo and 1/dn of the edges 10^(lo + k dn), for a first guess
    //        of a cell's bin.
    double *diag;
    double *dint;
    double *dhist;
    const double *hedges;
    int hbins, hfield;
    float hlo, hidn;
};

// Host helpers shared by the solver and the server (meso_api.hip).
constexpr size_t kAlign = 256;
inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline int pitch_of(int nx) { return (int)round_up((size_t)nx, 64); }
bool valid_grid(const mf_grid *g);
bool valid_materials(const mf_material *mat);
// conserved planes of a solve with these materials: 7 if the liquid reacts
int planes_of(const mf_material *mat);
bool valid_scheme(const mf_options *opt);
// bytes of one pitched state copy (nc planes), 256-byte rounded
size_t state_bytes(const mf_grid *g, int prec, int nc);
// Uniform rows per workgroup segment for one launch over n grids of
// nstrips[i] strips and ny[i] rows on a device of `cus` compute units (0: 256).
int seg_h_model(const int *nstrips, const int *ny, int n, int cus);
// The tail for one grid whose uniform model height is h, in precision mode
// prec (MF_FP*); updates h, and sets h2 = 0 when the grid keeps uniform
// segments.
void seg_taper(int nstrips, int ny, int cus, int prec, int &h, int &h2, int &tail_rows);
// Segments of one grid: h rows each, or (1 <= h2 < h, tail_rows > 0) h rows
// down to the last tail_rows or more rows, which get h2-row segments;
// uniform if the tail would not fit or exceed the launch's segment limit.
void set_segments(Desc &d, int ny, int h, int h2, int tail_rows);
int device_cus();
// Fill a descriptor for a solve whose workspace (control block + two state
// copies) starts at base.
void fill_desc(Desc &d, const mf_grid *g, const mf_material *mat, const mf_options *opt,
               char *base, int seg_h);

// Launchers (meso_kernels.hip).  All enqueue on `st` and return the launch
// status.  `prec` is kP64 / kPMix / kP32, `lim` the limiter id.
hipError_t launch_init_control(const Desc &d, double t, long long step, hipStream_t st);
hipError_t launch_prim_to_cons(const Desc &d, int prec, int dst, const double *prim,
                               hipStream_t st);
hipError_t launch_cons_from_f64(const Desc &d, int prec, int dst, const double *cons,
                                hipStream_t st);
hipError_t launch_reduce(const Desc &d, int prec, int src, hipStream_t st);
hipError_t launch_dt(const Desc &d, double cfl, double dx, double dy, double dt_fixed,
                     double t_end, hipStream_t st);
hipError_t launch_step(const Desc &d, int prec, int lim, int mode, int final_pass, int src,
                       hipStream_t st);
hipError_t launch_read_field(const Desc &d, int prec, int src, int field, double *out,
                             hipStream_t st);
// Diagnostics: out = (3 + nc) * nx doubles (pbar, rhobar, ubar, nc column sums);
// integrals from those column sums; a mass-weighted log-binned histogram.
hipError_t launch_columns(const Desc &d, int prec, int src, double *out, hipStream_t st);
hipError_t launch_integrals(const Desc &d, const double *cols, double *out, hipStream_t st);
hipError_t launch_histogram(const Desc &d, int prec, int src, int field, const double *edges,
                            int nbins, double m_ref, double dn, double *bins, hipStream_t st);
// One row (p_bar, rho_bar, u_bar; 3 * nx doubles) of a fused-averages record
// from the segment sums a recording step left at d.diag; NaN if the step was
// skipped.
hipError_t launch_diag_row(const Desc &d, double *row, hipStream_t st);
// One row of a fused-integrals record: the nc integrals (cell area times the
// workgroup sums at d.dint, added in workgroup order) and the time of the
// state; NaN if skipped.
hipError_t launch_int_row(const Desc &d, double *row, hipStream_t st);
// A fused-histogram row: zeroed before the recording step (hist_clear), then
// divided by m_ref * dn, or NaN if the step was skipped (hist_finish).
hipError_t launch_hist_clear(double *row, int nbins, hipStream_t st);
hipError_t launch_hist_finish(const Desc &d, double *row, int nbins, double m_ref_dn,
                              hipStream_t st);
// Many solves at once: descs/tiles are device arrays; tiles[b] = (solve index
// into descs, strip, segment, unused); every tile of one launch belongs to a
// solve whose liquid is `eos` and which has `nc` conserved planes (7: reactive).
hipError_t launch_batched_dt(const Desc *descs, int n, hipStream_t st);
hipError_t launch_batched_step(const Desc *descs, const int4 *tiles, int ntiles, int prec,
                               int lim, int eos, int nc, hipStream_t st);
// The FP32-bulk instantiations (meso_kernels_fast.hip) and the FP32 ones
// (meso_kernels_fp32.hip), inert liquids.
hipError_t launch_step_fast(const Desc &d, int lim, int mode, int final_pass, int src,
                            hipStream_t st);
hipError_t launch_batched_step_fast(const Desc *descs, const int4 *tiles, int ntiles, int lim,
                                    int eos, hipStream_t st);
hipError_t launch_step_fp32(const Desc &d, int lim, int mode, int final_pass, int src,
                            hipStream_t st);
hipError_t launch_batched_step_fp32(const Desc *descs, const int4 *tiles, int ntiles, int lim,
                                    int eos, hipStream_t st);
// Reactive solves (seven components): FP64 (meso_kernels_react.hip) and the
// FP32-bulk / FP32 modes (meso_kernels_react_fast.hip).
hipError_t launch_step_react(const Desc &d, int prec, int lim, int mode, int final_pass, int src,
                             hipStream_t st);
hipError_t launch_step_react_fast(const Desc &d, int prec, int lim, int mode, int final_pass,
                                  int src, hipStream_t st);
hipError_t launch_batched_step_react(const Desc *descs, const int4 *tiles, int ntiles, int prec,
                                     int lim, hipStream_t st);
hipError_t launch_batched_step_react_fast(const Desc *descs, const int4 *tiles, int ntiles,
                                          int prec, int lim, hipStream_t st);
// The fast FP64 mode, inert and reactive (meso_kernels_fast64.hip).
hipError_t launch_step_fast64(const Desc &d, int lim, int mode, int final_pass, int src,
                              hipStream_t st);
hipError_t launch_batched_step_fast64(const Desc *descs, const int4 *tiles, int ntiles, int lim,
                                      int eos, int nc, hipStream_t st);

}  // namespace meso
