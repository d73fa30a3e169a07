// meso_kernels.hip -- kernels of the FP64 mode (built with
// -ffp-contract=off: every operation rounds separately, as in the arithmetic
// contract), the small kernels around a step, and the launchers.

#include "meso_device.h"

namespace meso {

// ------------------------------------------------------------------------
// Small kernels around the step.

// Time step of the step about to run (one thread).  dt_fixed > 0 replaces the
// CFL bound cfl / s_max of the current state, but may not exceed it: a larger
// one latches a CFL violation (error bit 2) and the step is not taken.  t_end
// > 0 shortens the last step to land on t_end and turns later steps into
// no-ops.
__global__ void dt_kernel(Control *ctl, double cfl, double dx, double dy, double dt_fixed,
                          double t_end) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const long long n = ctl->step;
    if (ctl->err || (t_end > 0.0 && ctl->t >= t_end)) {
        ctl->skip = 1;
        return;
    }
    const double smax = __longlong_as_double((long long)ctl->smax_bits[n & 1]);
    if (!(smax > 0.0) || !(smax <= 1.0e300)) {
        ctl->err |= 1;
        ctl->skip = 1;
        return;
    }
    double dt = cfl / smax;
    if (dt_fixed > 0.0) {
        if (dt_fixed > dt) {
            ctl->err |= 2;
            ctl->skip = 1;
            return;
        }
        dt = dt_fixed;
    }
    const double t = ctl->t;
    double tn;
    if (t_end > 0.0 && t + dt >= t_end) {
        dt = t_end - t;
        tn = t_end;
    } else {
        tn = t + dt;
    }
    const double lx = dt / dx, ly = dt / dy;
    ctl->dt = dt;
    ctl->lam_x = lx;
    ctl->lam_y = ly;
    ctl->hl_x = 0.5 * lx;
    ctl->hl_y = 0.5 * ly;
    ctl->smax_bits[(n + 1) & 1] = 0ULL;
    ctl->step_exec = n;
    ctl->step = n + 1;
    ctl->t = tn;
    ctl->skip = 0;
}

// Time steps of many solves (one thread each, CFL steps, no end time).
__global__ void batched_dt_kernel(const Desc *descs, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const Desc &d = descs[k];
    Control *ctl = d.ctl;
    const long long s = ctl->step;
    if (ctl->err) {
        ctl->skip = 1;
        return;
    }
    const double smax = __longlong_as_double((long long)ctl->smax_bits[s & 1]);
    if (!(smax > 0.0) || !(smax <= 1.0e300)) {
        ctl->err |= 1;
        ctl->skip = 1;
        return;
    }
    const double dt = d.cfl / smax;
    const double lx = dt / d.dx, ly = dt / d.dy;
    ctl->dt = dt;
    ctl->lam_x = lx;
    ctl->lam_y = ly;
    ctl->hl_x = 0.5 * lx;
    ctl->hl_y = 0.5 * ly;
    ctl->smax_bits[(s + 1) & 1] = 0ULL;
    ctl->step_exec = s;
    ctl->step = s + 1;
    ctl->t = ctl->t + dt;
    ctl->skip = 0;
}

__global__ void init_control_kernel(Control *ctl, double t, long long step) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    ctl->t = t;
    ctl->dt = 0.0;
    ctl->lam_x = ctl->lam_y = ctl->hl_x = ctl->hl_y = 0.0;
    ctl->smax_bits[0] = ctl->smax_bits[1] = 0ULL;
    ctl->step = step;
    ctl->step_exec = step;
    ctl->skip = 0;
    ctl->err = 0;
}

// Primitive planes (dense, FP64) -> conserved state (pitched, storage type).
template <class S>
__global__ void prim_to_cons_kernel(Desc d, int dst_idx, const double *prim) {
    const long long N = (long long)d.nx * d.ny;
    S *dst = (S *)d.buf[dst_idx];
    const Mix<double> m = mix_of<double>(d);
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < N;
         k += (long long)gridDim.x * blockDim.x) {
        const double z = prim[k], r1 = prim[N + k], r2 = prim[2 * N + k];
        const double u = prim[3 * N + k], v = prim[4 * N + k], p = prim[5 * N + k];
        const double z2 = 1.0 - z;
        const double a1 = z * r1, a2 = z2 * r2;
        const double rho = a1 + a2;
        const double xi = z * d.g1 + z2 * d.g2;
        double eta;
        if (d.eos2 == 1) {
            double eta2, psi2;
            liquid_terms<double, false>(m, a2, z2, eta2, psi2);
            eta = z * d.h1 + eta2;
        } else {
            eta = z * d.h1 + z2 * d.h2;
        }
        const double E = (p * xi + eta) + 0.5 * (rho * (u * u + v * v));
        const int j = (int)(k / d.nx), i = (int)(k - (long long)j * d.nx);
        const long long o = (long long)j * d.pitch + i;
        dst[o] = (S)a1;
        dst[d.plane + o] = (S)a2;
        dst[2 * d.plane + o] = (S)(rho * u);
        dst[3 * d.plane + o] = (S)(rho * v);
        dst[4 * d.plane + o] = (S)E;
        dst[5 * d.plane + o] = (S)z;
        if (d.nc == 7) dst[6 * d.plane + o] = (S)(a2 * prim[6 * N + k]);   // z2 rho2 lambda
    }
}

template <class S>
__global__ void cons_from_f64_kernel(Desc d, int dst_idx, const double *cons) {
    const long long N = (long long)d.nx * d.ny;
    S *dst = (S *)d.buf[dst_idx];
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < N;
         k += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(k / d.nx), i = (int)(k - (long long)j * d.nx);
        const long long o = (long long)j * d.pitch + i;
        for (int c = 0; c < d.nc; ++c) dst[c * d.plane + o] = (S)cons[c * N + k];
    }
}

// CFL maximum of a state (no pointwise stage), into the slot of the current step.
template <class S, int FAST>
__global__ __launch_bounds__(kThreads) void reduce_kernel(Desc d, int src_idx, int slot) {
    const long long N = (long long)d.nx * d.ny;
    const S *src = (const S *)d.buf[src_idx];
    const Mix<S> ms = mix_of<S>(d);
    const S idx = (S)d.idx, idy = (S)d.idy;
    if (slot < 0) slot = (int)(d.ctl->step & 1);
    S smax = S(0);
    int bad = 0;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < N;
         k += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(k / d.nx), i = (int)(k - (long long)j * d.nx);
        const long long o = (long long)j * d.pitch + i;
        S q[6], w[6], r, rc2;
#pragma unroll
        for (int c = 0; c < 6; ++c) q[c] = src[c * d.plane + o];
        cons_to_prim<S, FAST, 6>(ms, q, w, r, rc2);
        const S c = Ar<S, FAST>::sqrt_(rc2 * r);
        const S s = fmax((fabs(w[2]) + c) * idx, (fabs(w[3]) + c) * idy);
        if (!(r > S(0)) || !(rc2 > S(0)) || !(s <= Ar<S, FAST>::big())) bad = 1;
        else smax = fmax(smax, s);
    }
    block_cfl_commit((double)smax, bad, d.ctl, slot);
}

// One field of the state as dense FP64 (conserved planes are widened, derived
// fields 6-10 use the closure in the storage type, the reaction fields 12-14
// the FP64 closure of the widened state).
template <class S>
__global__ void read_field_kernel(Desc d, int src_idx, int field, double *out) {
    const long long N = (long long)d.nx * d.ny;
    const S *src = (const S *)d.buf[src_idx];
    const Mix<S> ms = mix_of<S>(d);
    const Mix<double> md = mix_of<double>(d);
    const Rx<double> rx = rx_of<double>(d);
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < N;
         k += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(k / d.nx), i = (int)(k - (long long)j * d.nx);
        const long long o = (long long)j * d.pitch + i;
        if (field < 6 || field == MF_Z2RHO2LAM) {
            out[k] = (double)src[(field < 6 ? field : 6) * d.plane + o];
            continue;
        }
        if (field >= MF_LAMBDA) {
            double q[7];
#pragma unroll
            for (int c = 0; c < 7; ++c) q[c] = (double)src[c * d.plane + o];
            if (field == MF_LAMBDA) out[k] = q[6] / q[1];
            else if (field == MF_T2) out[k] = liquid_temperature(md, rx, q);
            else out[k] = heat_release(md, rx, q);
            continue;
        }
        S q[6], w[6], r, rc2;
#pragma unroll
        for (int c = 0; c < 6; ++c) q[c] = src[c * d.plane + o];
        cons_to_prim<S, false, 6>(ms, q, w, r, rc2);
        double v;
        switch (field) {
            case 6: v = (double)(q[0] + q[1]); break;
            case 7: v = (double)w[2]; break;
            case 8: v = (double)w[3]; break;
            case 9: v = (double)w[4]; break;
            default: v = (double)Ar<S, false>::sqrt_(rc2 * r); break;
        }
        out[k] = v;
    }
}

// ------------------------------------------------------------------------
// Diagnostics (Sec. 4.2 transverse averages, Sec. 4.5 mass-weighted PDFs).
// The closure is evaluated in FP64 on the stored state; every sum runs in a
// fixed order (increasing j inside a column, then increasing i), so the
// results do not depend on the launch geometry.

// Column pass: out[0..2][i] = pbar, rhobar, density-weighted ubar; out[3+c][i]
// = sum over the column of conserved component c.  A workgroup takes kColW
// columns in blocks of kColRows rows.  Its four waves load a block (all of a
// thread's rows issued before any is converted) and write each cell's
// components, pressure and z1rho1 + z2rho2 to LDS; then each group of kColW
// threads adds one of the column sums over the block's rows in increasing j.
// Every sum therefore runs in the order of one sequential pass down the
// column, while the per-cell work is spread over all the waves; the loads of
// the next block are issued before a block is converted.
constexpr int kColRows = 24;
constexpr int kColW = 32;
constexpr int kColThreads = 256;
constexpr int kColGroups = kColThreads / kColW;          // 8
constexpr int kColPerThread = kColRows / kColGroups;     // 3 rows per thread and block

template <class S, int NC>
__global__ __launch_bounds__(kColThreads) void column_kernel(Desc d, int src_idx, double *out) {
    // [row][quantity][column]; quantities 0..NC-1 the components, NC the
    // pressure, NC+1 the density
    __shared__ double sv[kColRows][NC + 2][kColW];
    __shared__ double fin[NC + 2][kColW];
    const int t = threadIdx.x;
    const int cl = t % kColW;
    const int g = t / kColW;
    const int i = blockIdx.x * kColW + cl;
    const bool in = i < d.nx;
    const S *src = (const S *)d.buf[src_idx];
    const Mix<double> m = mix_of<double>(d);
    // group g sums quantity qa (the pressure, the density, then the
    // components); with NC = 7 group 0 also sums component 6
    const int qa = g == 0 ? NC : (g == 1 ? NC + 1 : g - 2);
    double sa = 0.0, sb = 0.0;
    // a thread's rows of the block at j0, loaded into q; rows and columns
    // beyond the grid load its last row or column (always in bounds, never
    // used), so every load is issued unconditionally and the next block's
    // loads stay in flight while a block is converted
    const int ic = in ? i : d.nx - 1;
    auto issue = [&](int j0, double (&q)[kColPerThread][7]) {
#pragma unroll
        for (int u = 0; u < kColPerThread; ++u) {
            const int row = min(j0 + g + u * kColGroups, d.ny - 1);
            const long long o = (long long)row * d.pitch + ic;
#pragma unroll
            for (int c = 0; c < NC; ++c) q[u][c] = (double)src[c * d.plane + o];
            if constexpr (NC == 6) q[u][6] = 0.0;
        }
    };
    // convert the block at j0 into LDS and add it to the sums
    auto consume = [&](int j0, double (&q)[kColPerThread][7]) {
        const int nr = min(kColRows, d.ny - j0);
#pragma unroll
        for (int u = 0; u < kColPerThread; ++u) {
            const int r = g + u * kColGroups;
            if (in && r < nr) {
                double w[6], rr, rc2;
                cons_to_prim<double, false, 6>(m, q[u], w, rr, rc2);
#pragma unroll
                for (int c = 0; c < NC; ++c) sv[r][c][cl] = q[u][c];
                sv[r][NC][cl] = w[4];
                sv[r][NC + 1][cl] = q[u][0] + q[u][1];
            }
        }
        __syncthreads();
        if (in) {
            for (int r = 0; r < nr; ++r) {
                sa = sa + sv[r][qa][cl];
                if constexpr (NC == 7) {
                    if (g == 0) sb = sb + sv[r][6][cl];
                }
            }
        }
        __syncthreads();
    };
    // two register sets: block j1's loads are issued before block j0 is
    // converted and summed
    double bufA[kColPerThread][7], bufB[kColPerThread][7];
    issue(0, bufA);
    for (int j0 = 0; j0 < d.ny; j0 += 2 * kColRows) {
        const int j1 = j0 + kColRows;
        if (j1 < d.ny) issue(j1, bufB);
        consume(j0, bufA);
        if (j1 >= d.ny) break;
        if (j1 + kColRows < d.ny) issue(j1 + kColRows, bufA);
        consume(j1, bufB);
    }
    fin[qa][cl] = sa;
    if constexpr (NC == 7) {
        if (g == 0) fin[6][cl] = sb;
    }
    __syncthreads();
    if (!in) return;
    const long long n = d.nx;
    if (g == 0) out[i] = fin[NC][cl] / (double)d.ny;
    if (g == 1) out[n + i] = fin[NC + 1][cl] / (double)d.ny;
    if (g == 2) out[2 * n + i] = fin[2][cl] / fin[NC + 1][cl];
    for (int c = g; c < NC; c += kColGroups) out[(3 + c) * n + i] = fin[c][cl];
}

// Domain integrals from the column sums: thread c sums component c's column
// sums in increasing i (loads issued kColRows ahead of the sums).
__global__ void integrals_kernel(int nx, int nc, double area, const double *cols, double *out) {
    const int c = threadIdx.x;
    if (blockIdx.x != 0 || c >= nc) return;
    const double *s = cols + (long long)(3 + c) * nx;
    double tot = 0.0;
    int i = 0;
    for (; i + kColRows <= nx; i += kColRows) {
        double v[kColRows];
#pragma unroll
        for (int u = 0; u < kColRows; ++u) v[u] = s[i + u];
#pragma unroll
        for (int u = 0; u < kColRows; ++u) tot = tot + v[u];
    }
    for (; i < nx; ++i) tot = tot + s[i];
    out[c] = tot * area;
}

// One row of a fused-averages record: thread i adds column i's segment sums
// of a recording step in segment (row) order and forms p_bar = sum p / ny,
// rho_bar = sum rho / ny, u_bar = sum rho u / sum rho; a skipped step gives NaN.
__global__ void diag_row_kernel(const Control *ctl, const double *part, int nsegs, int nx,
                                int ny, double *row) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nx) return;
    const long long n = nx;   // 3 * nx may exceed the int range
    if (ctl->skip) {
        row[i] = row[n + i] = row[2 * n + i] = __longlong_as_double(0x7FF8000000000000LL);
        return;
    }
    double sp = 0.0, sr = 0.0, sm = 0.0;
    for (int g = 0; g < nsegs; ++g) {
        const double *b = part + g * 3 * n;
        sp = sp + b[i];
        sr = sr + b[n + i];
        sm = sm + b[2 * n + i];
    }
    row[i] = sp / (double)ny;
    row[n + i] = sr / (double)ny;
    row[2 * n + i] = sm / sr;
}

// One row of a fused-integrals record: block c adds plane c's workgroup sums
// (thread i takes workgroups i, i + 256, ... in order, then a fixed halving
// tree) and multiplies by the cell area; block 0 also writes the time of the
// state after the step at row[nc].  A skipped step gives NaN throughout.
__global__ __launch_bounds__(256) void int_row_kernel(const Control *ctl, const double *part,
                                                      int ntiles, int nc, double area,
                                                      double *row) {
    __shared__ double red[256];
    const int c = blockIdx.x, t = threadIdx.x;
    if (ctl->skip) {
        if (t == 0) row[c] = __longlong_as_double(0x7FF8000000000000LL);
        if (c == 0 && t == 0) row[nc] = __longlong_as_double(0x7FF8000000000000LL);
        return;
    }
    if (c == 0 && t == 0) row[nc] = ctl->t;
    double s = 0.0;
    for (int g = t; g < ntiles; g += 256) s = s + part[(long long)g * nc + c];
    red[t] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) red[t] = red[t] + red[t + h];
        __syncthreads();
    }
    if (t == 0) row[c] = red[0] * area;
}

// A fused-histogram row after its step: the bin masses divided by m_ref * dn
// (as mf_log_histogram does), or NaN if the step was skipped.
__global__ void hist_row_kernel(const Control *ctl, double *row, int n, double s) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) row[k] = ctl->skip ? __longlong_as_double(0x7FF8000000000000LL) : row[k] / s;
}

constexpr int kMaxBins = 1024;

// Mass-weighted histogram over log-spaced bins: bin a (edges[a] <= v <
// edges[a+1], v = pressure, density or the heat-release rate of a reactive
// liquid) collects z2 rho2 * area.  Per-workgroup
// LDS histograms, then one global atomic add per non-empty bin.
template <class S>
__global__ __launch_bounds__(kThreads) void histo_kernel(Desc d, int src_idx, int field,
                                                         const double *edges, int nbins,
                                                         double area, double *bins) {
    __shared__ double h[kMaxBins];
    __shared__ double e[kMaxBins + 1];
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) h[b] = 0.0;
    for (int b = threadIdx.x; b <= nbins; b += blockDim.x) e[b] = edges[b];
    __syncthreads();
    const S *src = (const S *)d.buf[src_idx];
    const Mix<double> m = mix_of<double>(d);
    const Rx<double> rx = rx_of<double>(d);
    const long long N = (long long)d.nx * d.ny;
    // grid-stride loop over the cells; (j, i) advance with the stride (one
    // carry, since the stride's column part is below nx) instead of a 64-bit
    // division per cell
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long k0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const int sj = (int)(stride / d.nx), si = (int)(stride - (long long)sj * d.nx);
    int j = (int)(k0 / d.nx), i = (int)(k0 - (long long)j * d.nx);
    for (long long k = k0; k < N; k += stride) {
        const long long o = (long long)j * d.pitch + i;
        double q[7], v;
        if (field == MF_QDOT) {
#pragma unroll
            for (int c = 0; c < 7; ++c) q[c] = (double)src[c * d.plane + o];
            v = heat_release(m, rx, q);
        } else {
            double w[6], r, rc2;
#pragma unroll
            for (int c = 0; c < 6; ++c) q[c] = (double)src[c * d.plane + o];
            cons_to_prim<double, false, 6>(m, q, w, r, rc2);
            v = (field == 6) ? (q[0] + q[1]) : w[4];
        }
        if (v >= e[0] && v < e[nbins]) {
            int a = 0, z = nbins;
            while (z - a > 1) {
                const int hh = (a + z) / 2;
                if (e[hh] <= v) a = hh;
                else z = hh;
            }
            atomicAdd(&h[a], q[1] * area);
        }
        i += si;
        j += sj;
        if (i >= d.nx) {
            i -= d.nx;
            ++j;
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += blockDim.x)
        if (h[b] != 0.0) atomicAdd(&bins[b], h[b]);
}

__global__ void fill_kernel(double *x, int n, double v) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) x[k] = v;
}

__global__ void scale_kernel(double *x, int n, double s) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) x[k] = x[k] / s;
}

// ------------------------------------------------------------------------
// Launchers.
static int grid_for(long long n) {
    long long g = (n + kThreads - 1) / kThreads;
    return (int)(g < 4096 ? (g < 1 ? 1 : g) : 4096);
}

hipError_t launch_init_control(const Desc &d, double t, long long step, hipStream_t st) {
    hipLaunchKernelGGL(init_control_kernel, dim3(1), dim3(64), 0, st, d.ctl, t, step);
    return hipGetLastError();
}

hipError_t launch_prim_to_cons(const Desc &d, int prec, int dst, const double *prim,
                               hipStream_t st) {
    const int g = grid_for((long long)d.nx * d.ny);
    if (prec == kP32)
        hipLaunchKernelGGL(prim_to_cons_kernel<float>, dim3(g), dim3(kThreads), 0, st, d, dst,
                           prim);
    else
        hipLaunchKernelGGL(prim_to_cons_kernel<double>, dim3(g), dim3(kThreads), 0, st, d, dst,
                           prim);
    return hipGetLastError();
}

hipError_t launch_cons_from_f64(const Desc &d, int prec, int dst, const double *cons,
                                hipStream_t st) {
    const int g = grid_for((long long)d.nx * d.ny);
    if (prec == kP32)
        hipLaunchKernelGGL(cons_from_f64_kernel<float>, dim3(g), dim3(kThreads), 0, st, d, dst,
                           cons);
    else
        hipLaunchKernelGGL(cons_from_f64_kernel<double>, dim3(g), dim3(kThreads), 0, st, d, dst,
                           cons);
    return hipGetLastError();
}

hipError_t launch_reduce(const Desc &d, int prec, int src, hipStream_t st) {
    const int g = grid_for((long long)d.nx * d.ny);
    // slot -1: the slot read by the next step, i.e. the parity of the
    // completed-step count held in the control block
    if (prec == kP32)
        hipLaunchKernelGGL((reduce_kernel<float, true>), dim3(g), dim3(kThreads), 0, st, d, src, -1);
    else if (prec == kPMix)
        hipLaunchKernelGGL((reduce_kernel<double, true>), dim3(g), dim3(kThreads), 0, st, d, src, -1);
    else
        hipLaunchKernelGGL((reduce_kernel<double, false>), dim3(g), dim3(kThreads), 0, st, d, src, -1);
    return hipGetLastError();
}

hipError_t launch_dt(const Desc &d, double cfl, double dx, double dy, double dt_fixed,
                     double t_end, hipStream_t st) {
    hipLaunchKernelGGL(dt_kernel, dim3(1), dim3(64), 0, st, d.ctl, cfl, dx, dy, dt_fixed, t_end);
    return hipGetLastError();
}

hipError_t launch_step(const Desc &d, int prec, int lim, int mode, int final_pass, int src,
                       hipStream_t st) {
    if (prec == kP64F) return launch_step_fast64(d, lim, mode, final_pass, src, st);
    if (d.nc == 7) return launch_step_react(d, prec, lim, mode, final_pass, src, st);
    if (prec == kP32) return launch_step_fp32(d, lim, mode, final_pass, src, st);
    if (prec == kPMix) return launch_step_fast(d, lim, mode, final_pass, src, st);
    if (lim == 1) launch_step_variants<double, double, false, 1, 6>(d, mode, final_pass, src, st);
    else launch_step_variants<double, double, false, 0, 6>(d, mode, final_pass, src, st);
    return hipGetLastError();
}

hipError_t launch_batched_dt(const Desc *descs, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(batched_dt_kernel, dim3((n + 63) / 64), dim3(64), 0, st, descs, n);
    return hipGetLastError();
}

hipError_t launch_batched_step(const Desc *descs, const int4 *tiles, int ntiles, int prec,
                               int lim, int eos, int nc, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (prec == kP64F) return launch_batched_step_fast64(descs, tiles, ntiles, lim, eos, nc, st);
    if (nc == 7) return launch_batched_step_react(descs, tiles, ntiles, prec, lim, st);
    if (prec == kP32) return launch_batched_step_fp32(descs, tiles, ntiles, lim, eos, st);
    if (prec == kPMix) return launch_batched_step_fast(descs, tiles, ntiles, lim, eos, st);
    launch_batched_variants<double, double, false, 6>(descs, tiles, ntiles, lim, eos, st);
    return hipGetLastError();
}

hipError_t launch_read_field(const Desc &d, int prec, int src, int field, double *out,
                             hipStream_t st) {
    const int g = grid_for((long long)d.nx * d.ny);
    if (prec == kP32)
        hipLaunchKernelGGL(read_field_kernel<float>, dim3(g), dim3(kThreads), 0, st, d, src,
                           field, out);
    else
        hipLaunchKernelGGL(read_field_kernel<double>, dim3(g), dim3(kThreads), 0, st, d, src,
                           field, out);
    return hipGetLastError();
}


hipError_t launch_columns(const Desc &d, int prec, int src, double *out, hipStream_t st) {
    const int g = (d.nx + kColW - 1) / kColW;
    void (*k)(Desc, int, double *);
    if (prec == kP32) k = d.nc == 7 ? column_kernel<float, 7> : column_kernel<float, 6>;
    else k = d.nc == 7 ? column_kernel<double, 7> : column_kernel<double, 6>;
    hipLaunchKernelGGL(k, dim3(g), dim3(kColThreads), 0, st, d, src, out);
    return hipGetLastError();
}

hipError_t launch_diag_row(const Desc &d, double *row, hipStream_t st) {
    hipLaunchKernelGGL(diag_row_kernel, dim3((d.nx + 255) / 256), dim3(256), 0, st, d.ctl, d.diag,
                       d.nsegs, d.nx, d.ny, row);
    return hipGetLastError();
}

hipError_t launch_int_row(const Desc &d, double *row, hipStream_t st) {
    hipLaunchKernelGGL(int_row_kernel, dim3(d.nc), dim3(256), 0, st, d.ctl, d.dint,
                       d.nstrips * d.nsegs, d.nc, d.dx * d.dy, row);
    return hipGetLastError();
}

hipError_t launch_hist_clear(double *row, int nbins, hipStream_t st) {
    hipLaunchKernelGGL(fill_kernel, dim3((nbins + 255) / 256), dim3(256), 0, st, row, nbins, 0.0);
    return hipGetLastError();
}

hipError_t launch_hist_finish(const Desc &d, double *row, int nbins, double m_ref_dn,
                              hipStream_t st) {
    hipLaunchKernelGGL(hist_row_kernel, dim3((nbins + 255) / 256), dim3(256), 0, st, d.ctl, row,
                       nbins, m_ref_dn);
    return hipGetLastError();
}

hipError_t launch_integrals(const Desc &d, const double *cols, double *out, hipStream_t st) {
    hipLaunchKernelGGL(integrals_kernel, dim3(1), dim3(64), 0, st, d.nx, d.nc, d.dx * d.dy, cols,
                       out);
    return hipGetLastError();
}

hipError_t launch_histogram(const Desc &d, int prec, int src, int field, const double *edges,
                            int nbins, double m_ref, double dn, double *bins, hipStream_t st) {
    if (nbins < 1 || nbins > kMaxBins) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fill_kernel, dim3((nbins + 255) / 256), dim3(256), 0, st, bins, nbins, 0.0);
    const int g = grid_for((long long)d.nx * d.ny);
    const double area = d.dx * d.dy;
    if (prec == kP32)
        hipLaunchKernelGGL(histo_kernel<float>, dim3(g), dim3(kThreads), 0, st, d, src, field,
                           edges, nbins, area, bins);
    else
        hipLaunchKernelGGL(histo_kernel<double>, dim3(g), dim3(kThreads), 0, st, d, src, field,
                           edges, nbins, area, bins);
    hipLaunchKernelGGL(scale_kernel, dim3((nbins + 255) / 256), dim3(256), 0, st, bins, nbins,
                       m_ref * dn);
    return hipGetLastError();
}

}  // namespace meso
