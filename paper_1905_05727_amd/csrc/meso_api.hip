// meso_api.hip -- host side of the C ABI declared in include/meso.h.
//
// Owns the device workspace layout (control block + two pitched state
// copies), enqueues the kernels of a step on the caller's stream and turns
// latched device errors into status codes at synchronising calls.

#include "meso.h"
#include "meso_internal.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

using meso::Control;
using meso::Desc;

namespace meso {

bool valid_grid(const mf_grid *g) {
    if (!g) return false;
    if (g->nx < 1 || g->ny < 1) return false;
    if (!(g->dx > 0.0) || !(g->dy > 0.0) || !isfinite(g->dx) || !isfinite(g->dy)) return false;
    const int32_t b[4] = {g->bc_xlo, g->bc_xhi, g->bc_ylo, g->bc_yhi};
    for (int i = 0; i < 4; ++i)
        if (b[i] != MF_BC_TRANSMISSIVE && b[i] != MF_BC_PERIODIC) return false;
    if ((g->bc_xlo == MF_BC_PERIODIC) != (g->bc_xhi == MF_BC_PERIODIC)) return false;
    if ((g->bc_ylo == MF_BC_PERIODIC) != (g->bc_yhi == MF_BC_PERIODIC)) return false;
    if (g->nx > (1 << 30) || g->ny > (1 << 30)) return false;
    if ((long long)g->nx * g->ny > (1LL << 40)) return false;
    return true;
}

bool valid_materials(const mf_material *mat) {
    if (!mat) return false;
    if (mat[0].reactive != 0 || (mat[1].reactive != 0 && mat[1].reactive != 1)) return false;
    if (mat[1].reactive) {
        const mf_material &m = mat[1];
        if (m.kind != MF_EOS_COCHRAN_CHAN || !(m.cv > 0.0) || !isfinite(m.cv) ||
            !(m.arr_C > 0.0) || !isfinite(m.arr_C) || !(m.arr_Ta >= 0.0) ||
            !isfinite(m.arr_Ta) || !(m.heat_Q >= 0.0) || !isfinite(m.heat_Q))
            return false;
    }
    for (int k = 0; k < 2; ++k) {
        if (mat[k].kind == MF_EOS_STIFFENED) {
            if (!(mat[k].gamma > 1.0) || !isfinite(mat[k].gamma) || !(mat[k].p_inf >= 0.0) ||
                !isfinite(mat[k].p_inf))
                return false;
        } else if (mat[k].kind == MF_EOS_COCHRAN_CHAN && k == 1) {
            const mf_material &m = mat[k];
            if (!(m.gamma0 > 0.0) || !(m.rho0 > 0.0) || !isfinite(m.gamma0) || !isfinite(m.A) ||
                !isfinite(m.B) || !isfinite(m.C) || !isfinite(m.D) || !isfinite(m.rho0) ||
                m.C == 1.0 || m.D == 1.0)
                return false;
        } else {
            return false;
        }
    }
    return true;
}

bool valid_scheme(const mf_options *opt) {
    if (!opt) return false;
    if (!(opt->cfl > 0.0) || !(opt->cfl <= 1.0)) return false;
    if (!(opt->z_floor >= 0.0) || !(opt->z_floor < 0.5)) return false;
    if (opt->limiter != MF_LIM_VANLEER && opt->limiter != MF_LIM_MINMOD) return false;
    if (opt->precision < MF_FP64 || opt->precision > MF_FP64_FAST) return false;
    return true;
}

int planes_of(const mf_material *mat) { return (mat && mat[1].reactive == 1) ? 7 : 6; }

size_t state_bytes(const mf_grid *g, int prec, int nc) {
    const size_t es = prec == MF_FP32 ? 4 : 8;
    return round_up((size_t)nc * pitch_of(g->nx) * (size_t)g->ny * es, kAlign);
}

int device_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

int seg_h_model(const int *nstrips, const int *ny, int n, int cus) {
    // Time per cell of a launch with h-row segments, fitted to kernel times
    // measured on MI355X over grids from 1000 x 4 to 8192 x 8192 in all three
    // precisions: the rows swept per row of output (every segment also sweeps
    // its 4 halo rows in x), times 1 + 1.45 CUs / workgroups, the imbalance of
    // few workgroups per compute unit at the end of the launch.  Ties go to
    // the taller segment.
    static const int kCand[] = {64, 48, 40, 32, 24, 20, 16, 12, 8, 6, 4, 2, 1};
    if (cus <= 0) cus = 256;
    int best = kCand[0];
    double best_t = -1.0;
    for (const int h : kCand) {
        double wgs = 0.0, rows = 0.0, swept = 0.0;
        for (int i = 0; i < n; ++i) {
            const int segs = (ny[i] + h - 1) / h;
            wgs += (double)nstrips[i] * segs;
            rows += (double)nstrips[i] * ny[i];
            swept += (double)nstrips[i] * (ny[i] + 4.0 * segs);
        }
        if (wgs <= 0.0) continue;
        const double t = swept / rows * (1.0 + 1.45 * cus / wgs);
        if (best_t < 0.0 || t < best_t) {
            best_t = t;
            best = h;
        }
    }
    return best;
}

void seg_taper(int nstrips, int ny, int cus, int prec, int &h, int &h2, int &tail_rows) {
    // Grids that the uniform model gives tall segments (>= 20 rows) do better
    // with taller segments still and a tail of short ones dispatched last:
    // rows h (32 or 64) down to a tail of h/5-row segments, about 3 workgroups
    // per compute unit in all (8 to 32 per strip, at most a fifth of the
    // rows).  Measured on MI355X against the uniform choice: 1.5-5 % faster
    // on 8192 x 8192, 4096 x 2048, 24000 x 313 and 24000 x 2000 in every mode
    // but one: the FP32-bulk kernel on grids under 32 strips (4 % slower on
    // 4096 x 2048), which keeps uniform segments.
    h2 = tail_rows = 0;
    if (h < 20) return;
    if (prec == MF_FP32_FP64ACC && nstrips < 32) return;
    if (cus <= 0) cus = 256;
    const int H = h >= 40 ? 64 : 32;
    const int t2 = H / 5;
    int n2 = (3 * cus + nstrips - 1) / nstrips;
    n2 = n2 < 8 ? 8 : (n2 > 32 ? 32 : n2);
    if ((long long)n2 * t2 * 5 > ny) return;
    h = H;
    h2 = t2;
    tail_rows = n2 * t2;
}

void set_segments(Desc &d, int ny, int h, int h2, int tail_rows) {
    if (h > ny) h = ny;   // one segment covers the strip (and ny + h - 1 stays in range)
    d.seg_h = d.seg_h2 = h;
    d.nsegs = d.seg_n1 = (ny + h - 1) / h;
    if (h2 < 1 || h2 >= h || tail_rows <= 0) return;
    const int n1 = (ny - tail_rows) / h;   // whole tall segments ahead of the tail
    if (n1 < 1) return;
    const long long n = (long long)n1 + (ny - (long long)n1 * h + h2 - 1) / h2;
    if (n > kMaxSegs) return;
    d.seg_n1 = n1;
    d.seg_h2 = h2;
    d.nsegs = (int)n;
}

void fill_desc(Desc &d, const mf_grid *g, const mf_material *mat, const mf_options *opt,
               char *base, int seg_h) {
    d.ctl = (Control *)base;
    d.diag = d.dint = d.dhist = nullptr;
    d.hedges = nullptr;
    d.hbins = d.hfield = 0;
    d.hlo = d.hidn = 0.0f;
    d.buf[0] = base + kAlign;
    d.nc = planes_of(mat);
    d.buf[1] = base + kAlign + state_bytes(g, opt->precision, d.nc);
    d.nx = g->nx;
    d.ny = g->ny;
    d.pitch = pitch_of(g->nx);
    d.plane = (long long)d.pitch * g->ny;
    d.bc_xlo = g->bc_xlo;
    d.bc_xhi = g->bc_xhi;
    d.bc_ylo = g->bc_ylo;
    d.bc_yhi = g->bc_yhi;
    d.nstrips = (g->nx + kTileW - 1) / kTileW;
    int h = seg_h, h2 = 0, tail = 0;
    if (h <= 0) {
        const char *fix = getenv("MESO_SEG_H");
        if (fix && atoi(fix) >= 1) {
            h = atoi(fix);
        } else {
            const int cus = device_cus();
            h = seg_h_model(&d.nstrips, &g->ny, 1, cus);
            seg_taper(d.nstrips, g->ny, cus, opt->precision, h, h2, tail);
        }
    }
    if (const char *env = getenv("MESO_SEG_TAPER")) {
        if (sscanf(env, "%d,%d", &h2, &tail) != 2) h2 = tail = 0;
    }
    // the segments of a strip are the launch's y dimension (at most 65535)
    const int min_h = (g->ny + kMaxSegs - 1) / kMaxSegs;
    if (h < min_h) h = min_h;
    set_segments(d, g->ny, h, h2, tail);
    d.dx = g->dx;
    d.dy = g->dy;
    d.cfl = opt->cfl;
    d.idx = 1.0 / g->dx;
    d.idy = 1.0 / g->dy;
    d.zlo = opt->z_floor;
    d.zhi = 1.0 - opt->z_floor;
    d.g1 = 1.0 / (mat[0].gamma - 1.0);
    d.h1 = (mat[0].gamma * mat[0].p_inf) * d.g1;
    d.eos2 = mat[1].kind;
    if (mat[1].kind == MF_EOS_COCHRAN_CHAN) {
        const mf_material &m = mat[1];
        d.ciG = 1.0 / m.gamma0;
        d.g2 = d.ciG;
        d.h2 = 0.0;
        d.cA = m.A;
        d.cB = m.B;
        d.cC = m.C;
        d.cD = m.D;
        d.crho0 = m.rho0;
        d.ckA = -m.A / (m.rho0 * (1.0 - m.C));
        d.ckB = m.B / (m.rho0 * (1.0 - m.D));
        d.cAC = m.A * m.C;
        d.cBD = m.B * m.D;
        d.cG0 = m.gamma0;
    } else {
        d.g2 = 1.0 / (mat[1].gamma - 1.0);
        d.h2 = (mat[1].gamma * mat[1].p_inf) * d.g2;
        d.ciG = d.cA = d.cB = d.cC = d.cD = d.crho0 = d.ckA = d.ckB = d.cAC = d.cBD = 0.0;
        d.cG0 = 0.0;
    }
    if (d.nc == 7) {
        d.rxcv = mat[1].cv;
        d.rxC = mat[1].arr_C;
        d.rxTa = mat[1].arr_Ta;
        d.rxQ = mat[1].heat_Q;
    } else {
        d.rxcv = d.rxC = d.rxTa = d.rxQ = 0.0;
    }
}

}  // namespace meso

namespace {

using meso::kAlign;
using meso::state_bytes;

struct EventPair {
    hipEvent_t a, b;
};

// One fused record: the caller's device rows, their number and the rows
// enqueued so far.
struct Record {
    double *rows;
    int64_t max, done;
    bool active() const { return rows && done < max; }
};

}  // namespace

struct mf_solver {
    Desc d;
    mf_grid grid;
    mf_material mat[2];
    mf_options opt;
    hipStream_t stream;
    void *ws;
    size_t ws_bytes;
    bool own_ws;
    long long host_step;  // completed steps once all enqueued work has run
    bool timing;
    std::vector<EventPair> ev;
    size_t ev_used;
    int device;           // HIP device current at creation
    // fused recording: library-owned partial sums and bin edges (allocated
    // on first use, freed by mf_destroy) and the caller's records
    double *rec_part;     // averages: 3 * nx column sums per segment
    double *int_part;     // integrals: nc sums per workgroup
    double *hist_edges;   // histogram: nbins + 1 edges (up to 1025)
    Record rec_avg, rec_int, rec_hist;
    int hist_bins, hist_field;
    double hist_mdn;      // m_ref * dn of the recorded histogram
    float hist_lo, hist_idn;   // lo and 1 / dn (the bin guess)
};

// Scratch of mf_integrals_noalloc: the column sums ((3 + nc) * nx doubles)
// followed by the nc integrals, in a file-scope device array (every device
// the library runs on holds its own copy until the process ends).  Host code
// never passes the array's name to a kernel: it is a host-side stand-in for
// the symbol, whose device address is looked up once per device.
static constexpr size_t kScratchDoubles = size_t(1) << 19;   // 4 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
double *scratch_ptr[kMaxDevices];   // device address of `scratch` on each device

// Device address of the scratch array on `device` (looked up on the first
// call for that device, with that device current; the caller's current
// device is restored).
int32_t scratch_on(int device, double **out) {
    if (device < 0 || device >= kMaxDevices) return MF_E_DEVICE;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[device]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) {
            (void)hipGetLastError();
            return MF_E_DEVICE;
        }
        if (cur != device && hipSetDevice(device) != hipSuccess) {
            (void)hipGetLastError();
            return MF_E_DEVICE;
        }
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return MF_E_DEVICE;
        }
        scratch_ptr[device] = (double *)p;
    }
    *out = scratch_ptr[device];
    return MF_OK;
}

}  // namespace

namespace {

int32_t dev_err(hipError_t e) { return e == hipSuccess ? MF_OK : MF_E_DEVICE; }

// Status of the latched device error bits (0 = none).
int32_t err_status(int err) {
    if (err & 2) return MF_E_CFL_VIOLATION;
    return err ? MF_E_NONFINITE_STATE : MF_OK;
}

// Index of the state copy that holds the state after `step` completed steps.
int state_index(const mf_solver *s, long long step) {
    return s->opt.fused ? (int)(step & 1) : 0;
}

int32_t read_control(mf_solver *s, Control *c) {
    if (hipStreamSynchronize(s->stream) != hipSuccess) return MF_E_DEVICE;
    if (hipMemcpy(c, s->d.ctl, sizeof(Control), hipMemcpyDeviceToHost) != hipSuccess)
        return MF_E_DEVICE;
    s->host_step = c->step;
    return MF_OK;
}

// After the state changed from the host: reset the control block and compute
// the CFL maximum of the new state for the next step.
int32_t restart(mf_solver *s, double t, long long step) {
    hipError_t e = meso::launch_init_control(s->d, t, step, s->stream);
    if (e == hipSuccess) e = meso::launch_reduce(s->d, s->opt.precision, state_index(s, step),
                                                 s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    s->host_step = step;
    return dev_err(e);
}

int32_t enqueue_step(mf_solver *s, double dt_fixed, double t_end) {
    hipError_t e = meso::launch_dt(s->d, s->opt.cfl, s->grid.dx, s->grid.dy, dt_fixed, t_end,
                                   s->stream);
    if (e != hipSuccess) return MF_E_DEVICE;
    const long long n = s->host_step;
    const int prec = s->opt.precision, lim = s->opt.limiter;
    const bool ra = s->opt.fused && s->rec_avg.active();
    const bool ri = s->opt.fused && s->rec_int.active();
    const bool rh = s->opt.fused && s->rec_hist.active();
    double *hrow = rh ? s->rec_hist.rows + s->rec_hist.done * (int64_t)s->hist_bins : nullptr;
    if (rh && meso::launch_hist_clear(hrow, s->hist_bins, s->stream) != hipSuccess)
        return MF_E_DEVICE;
    EventPair *ep = nullptr;
    if (s->timing) {
        if (s->ev_used == s->ev.size()) {
            EventPair p;
            if (hipEventCreate(&p.a) != hipSuccess) return MF_E_DEVICE;
            if (hipEventCreate(&p.b) != hipSuccess) return MF_E_DEVICE;
            s->ev.push_back(p);
        }
        ep = &s->ev[s->ev_used++];
        if (hipEventRecord(ep->a, s->stream) != hipSuccess) return MF_E_DEVICE;
    }
    if (s->opt.fused) {
        const int src = (int)(n & 1);
        s->d.diag = ra ? s->rec_part : nullptr;
        s->d.dint = ri ? s->int_part : nullptr;
        s->d.dhist = hrow;
        s->d.hedges = s->hist_edges;
        s->d.hbins = s->hist_bins;
        s->d.hfield = s->hist_field;
        s->d.hlo = s->hist_lo;
        s->d.hidn = s->hist_idn;
        e = meso::launch_step(s->d, prec, lim, (n & 1) ? meso::kYX : meso::kXY, 1, src,
                              s->stream);
    } else {
        // buffer 0 -> 1 in the first sweep, 1 -> 0 in the second
        const int first = (n & 1) ? meso::kY : meso::kX;
        const int second = (n & 1) ? meso::kX : meso::kY;
        e = meso::launch_step(s->d, prec, lim, first, 0, 0, s->stream);
        if (e == hipSuccess) e = meso::launch_step(s->d, prec, lim, second, 1, 1, s->stream);
    }
    if (e == hipSuccess && ep && hipEventRecord(ep->b, s->stream) != hipSuccess)
        e = hipErrorUnknown;
    if (e == hipSuccess && ra) {
        e = meso::launch_diag_row(
            s->d, s->rec_avg.rows + s->rec_avg.done * 3 * (int64_t)s->grid.nx, s->stream);
        ++s->rec_avg.done;
    }
    if (e == hipSuccess && ri) {
        e = meso::launch_int_row(s->d, s->rec_int.rows + s->rec_int.done * (int64_t)(s->d.nc + 1),
                                 s->stream);
        ++s->rec_int.done;
    }
    if (e == hipSuccess && rh) {
        e = meso::launch_hist_finish(s->d, hrow, s->hist_bins, s->hist_mdn, s->stream);
        ++s->rec_hist.done;
    }
    s->d.diag = s->d.dint = s->d.dhist = nullptr;
    if (e != hipSuccess) return MF_E_DEVICE;
    s->host_step = n + 1;
    return MF_OK;
}

// A library-owned device buffer of n doubles, allocated on first use.
int32_t alloc_once(double **p, size_t n) {
    if (*p) return MF_OK;
    if (hipMalloc(p, n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return MF_E_OUT_OF_MEMORY;
    }
    return MF_OK;
}

}  // namespace

extern "C" {

size_t mf_workspace_bytes(const mf_grid *grid, const mf_material mat[2], int32_t precision) {
    if (!meso::valid_grid(grid) || precision < MF_FP64 || precision > MF_FP64_FAST) return 0;
    if (mat && !meso::valid_materials(mat)) return 0;
    return kAlign + 2 * state_bytes(grid, precision, meso::planes_of(mat));
}

int32_t mf_create(const mf_grid *grid, const mf_material mat[2], const mf_options *opt,
                  void *dev_workspace, size_t ws_bytes, void *hip_stream, mf_solver **out) {
    if (!out) return MF_E_INVALID_ARG;
    *out = nullptr;
    if (!meso::valid_grid(grid) || !meso::valid_materials(mat) || !meso::valid_scheme(opt))
        return MF_E_INVALID_ARG;
    if (opt->fused != 0 && opt->fused != 1) return MF_E_INVALID_ARG;
    const size_t need = mf_workspace_bytes(grid, mat, opt->precision);
    if (dev_workspace && (ws_bytes < need || ((uintptr_t)dev_workspace % kAlign) != 0))
        return MF_E_INVALID_ARG;

    mf_solver *s = new (std::nothrow) mf_solver();
    if (!s) return MF_E_OUT_OF_MEMORY;
    s->grid = *grid;
    s->mat[0] = mat[0];
    s->mat[1] = mat[1];
    s->opt = *opt;
    s->stream = (hipStream_t)hip_stream;
    s->own_ws = dev_workspace == nullptr;
    s->ws_bytes = need;
    s->timing = false;
    s->ev_used = 0;
    if (hipGetDevice(&s->device) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return MF_E_DEVICE;
    }
    if (s->own_ws) {
        if (hipMalloc(&s->ws, need) != hipSuccess) {
            (void)hipGetLastError();
            delete s;
            return MF_E_OUT_OF_MEMORY;
        }
    } else {
        s->ws = dev_workspace;
    }
    Desc &d = s->d;
    meso::fill_desc(d, grid, mat, opt, (char *)s->ws, 0);

    hipError_t e = hipMemsetAsync(s->ws, 0, need, s->stream);
    if (e == hipSuccess) e = meso::launch_init_control(d, 0.0, 0, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        if (s->own_ws) (void)hipFree(s->ws);
        delete s;
        return MF_E_DEVICE;
    }
    s->host_step = 0;
    *out = s;
    return MF_OK;
}

static int32_t set_state(mf_solver *s, const double *host, bool prim) {
    if (!s || !host) return MF_E_INVALID_ARG;
    Control c;
    int32_t st = read_control(s, &c);
    if (st != MF_OK) return st;
    const size_t n = (size_t)s->grid.nx * s->grid.ny * s->d.nc;
    double *tmp = nullptr;
    if (hipMalloc(&tmp, n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return MF_E_OUT_OF_MEMORY;
    }
    hipError_t e = hipMemcpy(tmp, host, n * sizeof(double), hipMemcpyHostToDevice);
    const int dst = state_index(s, c.step);
    if (e == hipSuccess)
        e = prim ? meso::launch_prim_to_cons(s->d, s->opt.precision, dst, tmp, s->stream)
                 : meso::launch_cons_from_f64(s->d, s->opt.precision, dst, tmp, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return MF_E_DEVICE;
    return restart(s, c.t, c.step);
}

int32_t mf_set_primitive(mf_solver *s, const double *prim) { return set_state(s, prim, true); }

int32_t mf_set_conserved(mf_solver *s, const double *cons) { return set_state(s, cons, false); }

int32_t mf_set_time(mf_solver *s, double t, int64_t step) {
    if (!s || !isfinite(t) || step < 0) return MF_E_INVALID_ARG;
    Control c;
    int32_t st = read_control(s, &c);
    if (st != MF_OK) return st;
    const int from = state_index(s, c.step), to = state_index(s, step);
    if (from != to) {
        const size_t b = state_bytes(&s->grid, s->opt.precision, s->d.nc);
        if (hipMemcpyAsync(s->d.buf[to], s->d.buf[from], b, hipMemcpyDeviceToDevice,
                           s->stream) != hipSuccess)
            return MF_E_DEVICE;
    }
    return restart(s, t, step);
}

int32_t mf_step(mf_solver *s, double dt) {
    if (!s || !(dt == dt) || isinf(dt)) return MF_E_INVALID_ARG;
    return enqueue_step(s, dt > 0.0 ? dt : 0.0, 0.0);
}

int32_t mf_run_steps(mf_solver *s, int64_t nsteps) {
    if (!s || nsteps < 0) return MF_E_INVALID_ARG;
    for (int64_t i = 0; i < nsteps; ++i) {
        int32_t st = enqueue_step(s, 0.0, 0.0);
        if (st != MF_OK) return st;
    }
    return MF_OK;
}

int32_t mf_run_to_time(mf_solver *s, double t_end, int64_t max_steps, int64_t *steps_taken) {
    if (steps_taken) *steps_taken = 0;
    if (!s || !(t_end > 0.0) || !isfinite(t_end) || max_steps < 0) return MF_E_INVALID_ARG;
    Control c;
    int32_t st = read_control(s, &c);
    if (st != MF_OK) return st;
    if (c.err) return err_status(c.err);
    const long long start = c.step;
    long long chunk = 8;
    while (c.t < t_end && c.step - start < max_steps) {
        const long long left = max_steps - (c.step - start);
        const long long k = chunk < left ? chunk : left;
        for (long long i = 0; i < k; ++i) {
            st = enqueue_step(s, 0.0, t_end);
            if (st != MF_OK) return st;
        }
        st = read_control(s, &c);
        if (st != MF_OK) return st;
        if (c.err) break;
        if (chunk < 256) chunk *= 2;
    }
    if (steps_taken) *steps_taken = c.step - start;
    return err_status(c.err);
}

int32_t mf_sync(mf_solver *s) {
    if (!s) return MF_E_INVALID_ARG;
    Control c;
    int32_t st = read_control(s, &c);
    if (st != MF_OK) return st;
    return err_status(c.err);
}

int32_t mf_read_field(mf_solver *s, int32_t field, double *host_out, size_t count) {
    if (!s || !host_out || field < 0) return MF_E_INVALID_ARG;
    if (field > MF_C && !(s->d.nc == 7 && field >= MF_Z2RHO2LAM && field <= MF_QDOT))
        return MF_E_INVALID_ARG;
    const size_t n = (size_t)s->grid.nx * s->grid.ny;
    if (count != n) return MF_E_INVALID_ARG;
    Control c;
    int32_t st = read_control(s, &c);
    if (st != MF_OK) return st;
    if (c.err) return err_status(c.err);
    double *tmp = nullptr;
    if (hipMalloc(&tmp, n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return MF_E_OUT_OF_MEMORY;
    }
    hipError_t e = meso::launch_read_field(s->d, s->opt.precision, state_index(s, c.step), field,
                                           tmp, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) e = hipMemcpy(host_out, tmp, n * sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(tmp);
    return dev_err(e);
}

int32_t mf_read_conserved(mf_solver *s, double *host_out, size_t count) {
    if (!s || !host_out) return MF_E_INVALID_ARG;
    const size_t n = (size_t)s->grid.nx * s->grid.ny;
    const int nc = s->d.nc;
    if (count != (size_t)nc * n) return MF_E_INVALID_ARG;
    for (int f = 0; f < nc; ++f) {
        int32_t st = mf_read_field(s, f < 6 ? f : MF_Z2RHO2LAM, host_out + f * n, n);
        if (st != MF_OK) return st;
    }
    return MF_OK;
}

// Column sums of the current state into a temporary device array
// ((3 + nc) * nx, then room for the nc integrals).
static int32_t column_pass(mf_solver *s, double **cols_out) {
    Control c;
    int32_t st = read_control(s, &c);
    if (st != MF_OK) return st;
    if (c.err) return err_status(c.err);
    double *cols = nullptr;
    if (hipMalloc(&cols, sizeof(double) * ((3 + (size_t)s->d.nc) * s->grid.nx + 8)) !=
        hipSuccess) {
        (void)hipGetLastError();
        return MF_E_OUT_OF_MEMORY;
    }
    hipError_t e = meso::launch_columns(s->d, s->opt.precision, state_index(s, c.step), cols,
                                        s->stream);
    if (e != hipSuccess) {
        (void)hipFree(cols);
        return MF_E_DEVICE;
    }
    *cols_out = cols;
    return MF_OK;
}

int32_t mf_y_averages(mf_solver *s, double *p_bar, double *rho_bar, double *u_bar, size_t nx) {
    if (!s || !p_bar || !rho_bar || !u_bar || nx != (size_t)s->grid.nx) return MF_E_INVALID_ARG;
    double *cols = nullptr;
    int32_t st = column_pass(s, &cols);
    if (st != MF_OK) return st;
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) e = hipMemcpy(p_bar, cols, nx * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(rho_bar, cols + nx, nx * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(u_bar, cols + 2 * nx, nx * sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(cols);
    return dev_err(e);
}

int32_t mf_integrals(mf_solver *s, double *out, size_t count) {
    if (!s || !out || count != (size_t)s->d.nc) return MF_E_INVALID_ARG;
    double *cols = nullptr;
    int32_t st = column_pass(s, &cols);
    if (st != MF_OK) return st;
    double *res = cols + (3 + (size_t)s->d.nc) * s->grid.nx;
    hipError_t e = meso::launch_integrals(s->d, cols, res, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) e = hipMemcpy(out, res, count * sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(cols);
    return dev_err(e);
}

int32_t mf_integrals_noalloc(mf_solver *s, double *out, size_t count) {
    if (!s || !out || count != (size_t)s->d.nc) return MF_E_INVALID_ARG;
    const size_t ncols = (3 + (size_t)s->d.nc) * s->grid.nx;
    if (ncols + count > kScratchDoubles) return MF_E_INVALID_ARG;
    double *cols = nullptr;
    int32_t st = scratch_on(s->device, &cols);
    if (st != MF_OK) return st;
    Control c;
    st = read_control(s, &c);
    if (st != MF_OK) return st;
    if (c.err) return err_status(c.err);
    // every value of both regions is written by the kernels below: nothing to clear
    double *res = cols + ncols;
    hipError_t e = meso::launch_columns(s->d, s->opt.precision, state_index(s, c.step), cols,
                                        s->stream);
    if (e == hipSuccess) e = meso::launch_integrals(s->d, cols, res, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) e = hipMemcpy(out, res, count * sizeof(double), hipMemcpyDeviceToHost);
    return dev_err(e);
}

int32_t mf_log_histogram(mf_solver *s, int32_t field, double lo, double dn, int32_t nbins,
                         double m_ref, double *f_out) {
    if (!s || !f_out ||
        (field != MF_P && field != MF_RHO && !(field == MF_QDOT && s->d.nc == 7)) ||
        nbins < 1 || nbins > 1024 ||
        !(dn > 0.0) || !isfinite(lo) || !isfinite(dn) || !(m_ref > 0.0))
        return MF_E_INVALID_ARG;
    Control c;
    int32_t st = read_control(s, &c);
    if (st != MF_OK) return st;
    if (c.err) return err_status(c.err);
    std::vector<double> edges(nbins + 1);
    for (int32_t k = 0; k <= nbins; ++k) edges[k] = pow(10.0, lo + (double)k * dn);
    double *dev = nullptr;
    if (hipMalloc(&dev, sizeof(double) * (2 * (size_t)nbins + 1)) != hipSuccess) {
        (void)hipGetLastError();
        return MF_E_OUT_OF_MEMORY;
    }
    double *d_edges = dev, *d_bins = dev + nbins + 1;
    hipError_t e = hipMemcpy(d_edges, edges.data(), sizeof(double) * (nbins + 1),
                             hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = meso::launch_histogram(s->d, s->opt.precision, state_index(s, c.step), field, d_edges,
                                   nbins, m_ref, dn, d_bins, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) e = hipMemcpy(f_out, d_bins, sizeof(double) * nbins, hipMemcpyDeviceToHost);
    (void)hipFree(dev);
    return dev_err(e);
}

int32_t mf_get_time(mf_solver *s, double *t, int64_t *step, double *last_dt) {
    if (!s) return MF_E_INVALID_ARG;
    Control c;
    int32_t st = read_control(s, &c);
    if (st != MF_OK) return st;
    if (t) *t = c.t;
    if (step) *step = c.step;
    if (last_dt) *last_dt = c.dt;
    return err_status(c.err);
}

int32_t mf_enable_timing(mf_solver *s, int32_t enable) {
    if (!s) return MF_E_INVALID_ARG;
    if (hipStreamSynchronize(s->stream) != hipSuccess) return MF_E_DEVICE;
    s->timing = enable != 0;
    s->ev_used = 0;
    return MF_OK;
}

int32_t mf_kernel_time(mf_solver *s, double *total_ms, int64_t *launches) {
    if (!s) return MF_E_INVALID_ARG;
    if (hipStreamSynchronize(s->stream) != hipSuccess) return MF_E_DEVICE;
    double tot = 0.0;
    for (size_t i = 0; i < s->ev_used; ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, s->ev[i].a, s->ev[i].b) != hipSuccess) return MF_E_DEVICE;
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = (int64_t)s->ev_used;
    s->ev_used = 0;
    return MF_OK;
}

int32_t mf_launch_info(mf_solver *s, int64_t *workgroups, int32_t *threads, int32_t *tile_w,
                       int32_t *tile_h) {
    if (!s) return MF_E_INVALID_ARG;
    if (workgroups) *workgroups = (int64_t)s->d.nstrips * s->d.nsegs;
    if (threads) *threads = meso::kThreads;
    if (tile_w) *tile_w = meso::kTileW;
    if (tile_h) *tile_h = s->d.seg_h;
    return MF_OK;
}

int32_t mf_record_averages(mf_solver *s, double *dev_rows, int64_t max_rows) {
    if (!s) return MF_E_INVALID_ARG;
    if (!dev_rows) {   // stop recording; the rows written stay the caller's
        s->rec_avg.rows = nullptr;
        return MF_OK;
    }
    if (!s->opt.fused || max_rows < 1 || ((uintptr_t)dev_rows % sizeof(double)) != 0)
        return MF_E_INVALID_ARG;
    const int32_t st = alloc_once(&s->rec_part, 3 * (size_t)s->grid.nx * s->d.nsegs);
    if (st != MF_OK) return st;
    s->rec_avg = Record{dev_rows, max_rows, 0};
    return MF_OK;
}

int32_t mf_record_integrals(mf_solver *s, double *dev_rows, int64_t max_rows) {
    if (!s) return MF_E_INVALID_ARG;
    if (!dev_rows) {
        s->rec_int.rows = nullptr;
        return MF_OK;
    }
    if (!s->opt.fused || max_rows < 1 || ((uintptr_t)dev_rows % sizeof(double)) != 0)
        return MF_E_INVALID_ARG;
    const int32_t st =
        alloc_once(&s->int_part, (size_t)s->d.nc * s->d.nstrips * (size_t)s->d.nsegs);
    if (st != MF_OK) return st;
    s->rec_int = Record{dev_rows, max_rows, 0};
    return MF_OK;
}

int32_t mf_record_histogram(mf_solver *s, int32_t field, double lo, double dn, int32_t nbins,
                            double m_ref, double *dev_rows, int64_t max_rows) {
    if (!s) return MF_E_INVALID_ARG;
    if (!dev_rows) {
        s->rec_hist.rows = nullptr;
        return MF_OK;
    }
    if (!s->opt.fused || max_rows < 1 || ((uintptr_t)dev_rows % sizeof(double)) != 0 ||
        (field != MF_P && field != MF_RHO && !(field == MF_QDOT && s->d.nc == 7)) ||
        nbins < 1 || nbins > 1024 || !(dn > 0.0) || !isfinite(lo) || !isfinite(dn) ||
        !(m_ref > 0.0))
        return MF_E_INVALID_ARG;
    int32_t st = alloc_once(&s->hist_edges, 1025);
    if (st != MF_OK) return st;
    // the same edges as mf_log_histogram; the stream may still be reading
    // the previous ones
    std::vector<double> edges(nbins + 1);
    for (int32_t k = 0; k <= nbins; ++k) edges[k] = pow(10.0, lo + (double)k * dn);
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess)
        e = hipMemcpy(s->hist_edges, edges.data(), sizeof(double) * (nbins + 1),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        s->rec_hist.rows = nullptr;
        return dev_err(e);
    }
    s->hist_bins = nbins;
    s->hist_field = field;
    s->hist_mdn = m_ref * dn;
    s->hist_lo = (float)lo;
    s->hist_idn = (float)(1.0 / dn);
    s->rec_hist = Record{dev_rows, max_rows, 0};
    return MF_OK;
}

int32_t mf_recorded_rows(mf_solver *s, int64_t *rows) {
    if (!s || !rows) return MF_E_INVALID_ARG;
    *rows = s->rec_avg.done;
    return MF_OK;
}

int32_t mf_recorded_counts(mf_solver *s, int64_t counts[3]) {
    if (!s || !counts) return MF_E_INVALID_ARG;
    counts[0] = s->rec_avg.done;
    counts[1] = s->rec_int.done;
    counts[2] = s->rec_hist.done;
    return MF_OK;
}

int32_t mf_destroy(mf_solver *s) {
    if (!s) return MF_E_INVALID_ARG;
    hipError_t e = hipStreamSynchronize(s->stream);
    if (s->rec_part) (void)hipFree(s->rec_part);
    if (s->int_part) (void)hipFree(s->int_part);
    if (s->hist_edges) (void)hipFree(s->hist_edges);
    for (auto &p : s->ev) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    if (s->own_ws) (void)hipFree(s->ws);
    delete s;
    return dev_err(e);
}

const char *mf_status_str(int32_t status) {
    switch (status) {
        case MF_OK: return "ok";
        case MF_E_INVALID_ARG: return "invalid argument";
        case MF_E_OUT_OF_MEMORY: return "out of device memory";
        case MF_E_NONFINITE_STATE: return "non-finite or non-physical state";
        case MF_E_CFL_VIOLATION: return "time step above the CFL bound of the state";
        case MF_E_DEVICE: return "HIP runtime error";
        case MF_E_NOT_READY: return "not ready";
        case MF_E_BUSY: return "busy";
        default: return "unknown status";
    }
}

const char *mf_version(void) { return "meso 0.1 gfx950"; }

}  // extern "C"
