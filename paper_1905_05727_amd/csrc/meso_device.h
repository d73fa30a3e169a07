// meso_device.h -- device code of the two-fluid finite-volume update,
// included by the kernel translation units: meso_kernels.hip and
// meso_kernels_react.hip (FP64 mode, built without floating-point
// contraction), meso_kernels_fast.hip and meso_kernels_react_fast.hip
// (FP32-bulk and FP32 modes, built with contraction).
//
// Equations: Eq. (1) (Sec. 2.1) -- partial densities, momentum, total energy,
// non-conservative advection of the air volume fraction z1, and for a
// reactive liquid the reactant mass z2 rho2 lambda -- with the
// pressure-equilibrium closure of Sec. 2.1, stiffened-gas phases (Eq. (2)
// with constant reference terms) or a Cochran-Chan liquid (Eqs. (2)-(4),
// Sec. 2.2), and Arrhenius kinetics (Eq. (6)) at the liquid temperature of
// Eq. (5).  Scheme of Sec. 3:
// MUSCL-Hancock in primitive variables, van Leer or minmod slopes, HLLC flux
// with the HLLC-consistent interface velocity for the z1 term, dimensionally
// split sweeps (x then y on even steps, y then x on odd ones), CFL time step
// and the pointwise stage of the Strang split (z1 clamp; reaction half-steps).
//
// Data layout in HBM: structure of arrays, 6 planes (z1 rho1, z2 rho2, rho u,
// rho v, rho E, z1) -- 7 with the reactant mass z2 rho2 lambda of a reactive
// liquid -- rows padded to a multiple of 64 elements; two state copies used as
// ping-pong buffers.  NC (6 or 7) is the number of conserved components, a
// template parameter so that the inert kernels carry no seventh component.
// EOS (0 stiffened-gas liquid, 1 Cochran-Chan liquid) is a template parameter
// of the step kernels for the same reason: the water kernels carry neither
// the pow of the Cochran-Chan reference curves nor its registers.  EOS = -1
// (the small kernels) selects the liquid at run time from the descriptor.
//
// Step kernel: a workgroup of 256 threads (4 wave64) owns a strip of 256
// columns (252 written + 2 halo columns per side) and marches down a segment
// of rows.  The x sweep of a row exchanges primitives, face states and fluxes
// between neighbouring threads through LDS; the y sweep is a per-thread
// rolling window held in registers (no exchange at all).  A fused step runs
// both sweeps in one pass over the segment, so the state is read and written
// once per step; the pointwise stage and the next step's CFL maximum are
// computed in the epilogue from the values about to be stored, and a
// recording step also sums the transverse averages of Sec. 4.2 there.
//
// Precision is a template parameter of the same code: S is the storage /
// accumulation type, R the type of reconstruction, predictor and Riemann
// solver.  FP64 (S = R = double) follows the arithmetic contract operation
// by operation (no contraction, IEEE division and square root).  The FP32
// flux path uses the hardware reciprocal and square root.

#pragma once

#include "meso_internal.h"

#include <float.h>

namespace meso {

// ------------------------------------------------------------------------
// Arithmetic policies, by level FAST.  Ar<double, 0>: IEEE division and
// square root (the FP64 mode, bit-compatible with the arithmetic contract; the
// two powers of the Cochran-Chan reference curves share one logarithm,
// v^-C = exp(-C ln v), a few ulp from a correctly rounded pow).
// Ar<double, 1>: hardware reciprocal refined by one Newton step and the
// hardware square root (the FP64 closure of the FP32-bulk mode).
// Ar<double, 2>: the fast FP64 mode -- reciprocal and reciprocal square root
// from the hardware seeds (about 23 correct bits) refined by the second-order
// series of 1/(1 - e) and (1 - e)^(-1/2) in the seed's residual e (error of
// order e^3, below the rounding), so every result is within about one ulp of
// the correctly rounded one at under half the instructions of the IEEE
// sequences.  Ar<float, *>: hardware reciprocal and square root.
template <class T, int FAST> struct Ar;
template <> struct Ar<double, 0> {
    // v^-C and v^-D of the Cochran-Chan reference curves
    static __device__ __forceinline__ void pw(double v, double C, double D, double &vc,
                                              double &vd) {
        const double l = log(v);
        vc = exp(-C * l);
        vd = exp(-D * l);
    }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static __device__ __forceinline__ double rcp(double a) { return 1.0 / a; }
    static __device__ __forceinline__ double sqrt_(double a) { return __builtin_sqrt(a); }
    static __device__ __forceinline__ double big() { return 1.0e300; }
    static __device__ __forceinline__ double ex(double a) { return exp(a); }
};
template <> struct Ar<double, 1> {
    static __device__ __forceinline__ void pw(double v, double C, double D, double &vc,
                                              double &vd) {
        const double l = log(v);
        vc = exp(-C * l);
        vd = exp(-D * l);
    }
    static __device__ __forceinline__ double rcp(double a) {
        const double r = __builtin_amdgcn_rcp(a);
        const double e = __builtin_fma(-a, r, 1.0);
        return __builtin_fma(r, e, r);
    }
    static __device__ __forceinline__ double div(double a, double b) { return a * rcp(b); }
    static __device__ __forceinline__ double sqrt_(double a) { return __builtin_amdgcn_sqrt(a); }
    static __device__ __forceinline__ double rsq(double a) { return __builtin_amdgcn_rsq(a); }
    static __device__ __forceinline__ double big() { return 1.0e300; }
    static __device__ __forceinline__ double ex(double a) { return exp(a); }
};
template <> struct Ar<double, 2> {
    static __device__ __forceinline__ void pw(double v, double C, double D, double &vc,
                                              double &vd) {
        const double l = log(v);
        vc = exp(-C * l);
        vd = exp(-D * l);
    }
    // 1/a from the seed r (relative error |e| < 2^-22, e = 1 - a r):
    // 1/a = r / (1 - e) = r (1 + e + e^2) + O(e^3)
    static __device__ __forceinline__ double rcp(double a) {
        const double r = __builtin_amdgcn_rcp(a);
        const double e = __builtin_fma(-a, r, 1.0);
        return __builtin_fma(r, __builtin_fma(e, e, e), r);
    }
    static __device__ __forceinline__ double div(double a, double b) { return a * rcp(b); }
    // 1/sqrt(a) from the seed y (e = 1 - a y^2):
    // 1/sqrt(a) = y (1 - e)^(-1/2) = y (1 + e/2 + 3 e^2/8) + O(e^3)
    static __device__ __forceinline__ double rsq(double a) {
        const double y = __builtin_amdgcn_rsq(a);
        const double e = __builtin_fma(-(a * y), y, 1.0);
        return __builtin_fma(y, e * __builtin_fma(e, 0.375, 0.5), y);
    }
    // sqrt(a) = a / sqrt(a), corrected by the residual a - s^2.  For a > 0
    // and finite only (0 gives NaN): the callers flag a non-positive a anyway
    static __device__ __forceinline__ double sqrt_(double a) {
        const double y = rsq(a);
        const double s = a * y;
        return __builtin_fma(__builtin_fma(-s, s, a), 0.5 * y, s);
    }
    static __device__ __forceinline__ double big() { return 1.0e300; }
    static __device__ __forceinline__ double ex(double a) { return exp(a); }
};
template <int FAST> struct Ar<float, FAST> {
    static __device__ __forceinline__ void pw(float v, float C, float D, float &vc, float &vd) {
        const float l = __builtin_amdgcn_logf(v);        // log2 v
        vc = __builtin_amdgcn_exp2f(-C * l);
        vd = __builtin_amdgcn_exp2f(-D * l);
    }
    static __device__ __forceinline__ float div(float a, float b) {
        return a * __builtin_amdgcn_rcpf(b);
    }
    static __device__ __forceinline__ float rcp(float a) { return __builtin_amdgcn_rcpf(a); }
    static __device__ __forceinline__ float sqrt_(float a) { return __builtin_amdgcn_sqrtf(a); }
    static __device__ __forceinline__ float rsq(float a) { return __builtin_amdgcn_rsqf(a); }
    static __device__ __forceinline__ float big() { return FLT_MAX; }
    static __device__ __forceinline__ float ex(float a) {   // e^a = 2^(a log2 e)
        return __builtin_amdgcn_exp2f(a * 1.44269504088896341f);
    }
};

// Mixture constants: every phase in the Mie-Grueneisen form of Eq. (2),
// rho_k e_k = phi_k(rho_k) + p / Gamma_k, so that rho e = p xi + eta with
// xi = sum z_k / Gamma_k and eta = sum z_k phi_k.  g = 1/Gamma; h = phi of a
// stiffened gas (constant); a Cochran-Chan liquid (eos2 = 1) has a density
// dependent phi (Eqs. (3)-(4)).
template <class T> struct Mix {
    T g1, g2, h1, h2;
    int eos2;
    T A, B, C, D, rho0, iG, kA, kB, AC, BD;
};

template <class T> __device__ __forceinline__ Mix<T> mix_of(const Desc &d) {
    Mix<T> m;
    m.g1 = (T)d.g1; m.g2 = (T)d.g2; m.h1 = (T)d.h1; m.h2 = (T)d.h2;
    m.eos2 = d.eos2;
    m.A = (T)d.cA; m.B = (T)d.cB; m.C = (T)d.cC; m.D = (T)d.cD; m.rho0 = (T)d.crho0;
    m.iG = (T)d.ciG; m.kA = (T)d.ckA; m.kB = (T)d.ckB; m.AC = (T)d.cAC; m.BD = (T)d.cBD;
    return m;
}

// Single-step Arrhenius kinetics of the reactive liquid (Eq. (6), Table 3)
// and the constants of its temperature (Eq. (5)): Gamma_0 and c_v.
template <class T> struct Rx {
    T C, Ta, Q, G0, cv;
};

template <class T> __device__ __forceinline__ Rx<T> rx_of(const Desc &d) {
    Rx<T> x;
    x.C = (T)d.rxC; x.Ta = (T)d.rxTa; x.Q = (T)d.rxQ; x.G0 = (T)d.cG0; x.cv = (T)d.rxcv;
    return x;
}

// Cochran-Chan liquid at partial density a2 and volume fraction z2:
// eta2 = z2 phi(rho2) and psi2 = z2 rho2 phi'(rho2), the term the density
// dependence of phi adds to the frozen sound speed
// rho c^2 = (p (1 + xi) + eta - psi) / xi.
template <class T, int FAST>
__device__ __forceinline__ void liquid_terms(const Mix<T> &m, T a2, T z2, T &eta2, T &psi2) {
    const T rho2 = Ar<T, FAST>::div(a2, z2);
    const T v = Ar<T, FAST>::div(m.rho0, rho2);
    T vc, vd;
    Ar<T, FAST>::pw(v, m.C, m.D, vc, vd);
    const T pref = m.A * vc - m.B * vd;
    const T eref = m.kA * (v * vc - T(1)) + m.kB * (v * vd - T(1));
    const T rdpref = m.AC * vc - m.BD * vd;
    const T phi = rho2 * eref - pref * m.iG;
    const T rphi = (rho2 * eref + pref) - rdpref * m.iG;
    eta2 = z2 * phi;
    psi2 = z2 * rphi;
}

// Ghost-cell index map: transmissive copies the edge cell, periodic wraps.
__device__ __forceinline__ int map_idx(int i, int n, int bc_lo, int bc_hi) {
    if (i < 0) return bc_lo ? ((i % n) + n) % n : 0;
    if (i >= n) return bc_hi ? i % n : n - 1;
    return i;
}

// ------------------------------------------------------------------------
// Closure (Sec. 2.1): sweep-frame conserved q = (a1, a2, mn, mt, E, z) to
// primitives w = (a1, a2, un, ut, p, z), 1/rho and rho c^2; with NC = 7 also
// q[6] = z2 rho2 lambda to w[6] = lambda, the liquid's unreacted mass fraction.
template <int EOS, class T> __device__ __forceinline__ bool is_cc(const Mix<T> &m) {
    return EOS < 0 ? m.eos2 == 1 : EOS == 1;
}

template <class S, int FAST, int NC, int EOS = -1>
__device__ __forceinline__ void cons_to_prim(const Mix<S> &m, const S q[NC], S w[NC], S &r,
                                             S &rc2) {
    const S rho = q[0] + q[1];
    const S z = q[5];
    const S z2 = S(1) - z;
    const S xi = z * m.g1 + z2 * m.g2;
    S eta, psi = S(0);
    if (is_cc<EOS>(m)) {
        S eta2;
        liquid_terms<S, FAST>(m, q[1], z2, eta2, psi);
        eta = z * m.h1 + eta2;
    } else {
        eta = z * m.h1 + z2 * m.h2;
    }
    S ixi;
    if constexpr (FAST) {   // one reciprocal for both 1/rho and 1/xi
        const S inv = Ar<S, FAST>::rcp(rho * xi);
        r = xi * inv;
        ixi = rho * inv;
    } else {
        r = Ar<S, FAST>::rcp(rho);
        ixi = Ar<S, FAST>::rcp(xi);
    }
    const S un = q[2] * r;
    const S ut = q[3] * r;
    const S ke = S(0.5) * (q[2] * un + q[3] * ut);
    const S rhoe = q[4] - ke;
    const S p = (rhoe - eta) * ixi;
    if (is_cc<EOS>(m)) rc2 = ((p * (S(1) + xi) + eta) - psi) * ixi;
    else rc2 = (p * (S(1) + xi) + eta) * ixi;
    w[0] = q[0]; w[1] = q[1]; w[2] = un; w[3] = ut; w[4] = p; w[5] = z;
    if constexpr (NC == 7) w[6] = Ar<S, FAST>::div(q[6], q[1]);
}

// Slope limiter (Sec. 3): a backward, b forward difference.  The van Leer
// division is needed only where a b > 0.  In the FP32 modes a wave in which
// no lane needs it (a region at rest or a uniform state) skips it; the FP64
// kernel stays branch-free, which keeps its six independent IEEE divisions
// interleaved (it is latency bound at 2 waves per SIMD).
template <class R, int FAST, int LIM>
__device__ __forceinline__ R limit(R a, R b) {
    const R ab = a * b;
    if (LIM == 1) {
        const R s = (a > R(0)) ? fmin(a, b) : fmax(a, b);
        return (ab > R(0)) ? s : R(0);
    }
    if constexpr (!FAST) {   // FP64: branch-free (keeps the divisions interleaved)
        const R v = Ar<R, FAST>::div(ab + ab, a + b);
        return (ab > R(0)) ? v : R(0);
    }
    R s = R(0);
    if (__builtin_amdgcn_ballot_w64(ab > R(0)) != 0) {
        const R v = Ar<R, FAST>::div(ab + ab, a + b);
        s = (ab > R(0)) ? v : R(0);
    }
    return s;
}

// MUSCL reconstruction and Hancock half step in primitive variables.
template <class R, int FAST, int LIM, int NC>
__device__ __forceinline__ void face_states(const R wm[NC], const R w0[NC], const R wp[NC], R r,
                                            R rc2, R hl, R wl[NC], R wh[NC]) {
    R d[NC], s[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) d[c] = limit<R, FAST, LIM>(w0[c] - wm[c], wp[c] - w0[c]);
    const R un = w0[2];
    s[0] = hl * (un * d[0] + w0[0] * d[2]);
    s[1] = hl * (un * d[1] + w0[1] * d[2]);
    s[2] = hl * (un * d[2] + r * d[4]);
    s[3] = hl * (un * d[3]);
    s[4] = hl * (un * d[4] + rc2 * d[2]);
    s[5] = hl * (un * d[5]);
    if constexpr (NC == 7) s[6] = hl * (un * d[6]);   // lambda is advected
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        wl[c] = (w0[c] - R(0.5) * d[c]) - s[c];
        wh[c] = (w0[c] + R(0.5) * d[c]) - s[c];
    }
}

// Sweep-side state of a Riemann problem.  side_eval fills what the wave
// speeds need -- primitives, the mixture terms xi and eta, the normal
// momentum U[2] -- and returns the sound speed; side_finish adds the total
// energy, the other conserved components U and the fluxes F (5 inert, a 6th
// for the reactant mass z2 rho2 lambda when NC = 7), and is evaluated only for
// the side(s) a face's flux uses.
template <class R, int NC> struct Side {
    R rho, un, ut, p, z, xi, eta, E;
    R a1, a2, lam;       // partial densities z1 rho1, z2 rho2; lambda (NC = 7)
    R U[NC - 1], F[NC - 1];
};

template <class R, int FAST, int NC, int EOS>
__device__ __forceinline__ void side_eval(const Mix<R> &m, const R w[NC], Side<R, NC> &s,
                                          R &c) {
    const R rho = w[0] + w[1];
    const R un = w[2], ut = w[3], p = w[4], z = w[5];
    const R z2 = R(1) - z;
    const R xi = z * m.g1 + z2 * m.g2;
    R eta, num;
    if (is_cc<EOS>(m)) {
        R eta2, psi2;
        liquid_terms<R, FAST>(m, w[1], z2, eta2, psi2);
        eta = z * m.h1 + eta2;
        num = (p * (R(1) + xi) + eta) - psi2;
    } else {
        eta = z * m.h1 + z2 * m.h2;
        num = p * (R(1) + xi) + eta;
    }
    if constexpr (FAST) c = num * Ar<R, FAST>::rsq(num * (xi * rho));   // sqrt(num / (xi rho))
    else c = Ar<R, FAST>::sqrt_(Ar<R, FAST>::div(num, xi * rho));
    s.rho = rho; s.un = un; s.ut = ut; s.p = p; s.z = z; s.xi = xi; s.eta = eta;
    s.a1 = w[0]; s.a2 = w[1];
    s.U[2] = rho * un;
    if constexpr (NC == 7) s.lam = w[6];
}

template <class R, int NC> __device__ __forceinline__ void side_finish(Side<R, NC> &s) {
    const R E = (s.p * s.xi + s.eta) + R(0.5) * (s.rho * (s.un * s.un + s.ut * s.ut));
    const R mn = s.U[2];
    s.E = E;
    s.U[0] = s.a1; s.U[1] = s.a2; s.U[3] = s.rho * s.ut; s.U[4] = E;
    s.F[0] = s.a1 * s.un;
    s.F[1] = s.a2 * s.un;
    s.F[2] = mn * s.un + s.p;
    s.F[3] = mn * s.ut;
    s.F[4] = (E + s.p) * s.un;
    if constexpr (NC == 7) {
        s.U[5] = s.a2 * s.lam;
        s.F[5] = s.U[5] * s.un;
    }
}

// Star-state flux F* = F + S (U* - U) of side k with wave speed S, contact
// speed S*.  KV (the fast FP64 and FP32 kernels): rearranged so that every
// component carried with the flow (partial densities, tangential momentum,
// reactant mass, the volume flux of z) is kv U with kv = d S* / (S - S*),
// d = S - u, the star state's volume flux velocity (0 exactly at S* = 0);
// normal momentum p + rho (d (S* - u) + kv S*), energy kv E + p u + S (S* - u)
// (chi rho S* + p / (S - S*)), chi = d / (S - S*).  Equal in exact arithmetic
// to the direct form, with fewer operations; the FP32-bulk kernel measured
// slower with it and keeps the direct form.
template <class R, int FAST, int NC, bool KV = false>
__device__ __forceinline__ void star_flux(const Side<R, NC> &k, R S, R Ss, R out[NC + 1]) {
    const R d = S - k.un;
    if constexpr (FAST != 0 && KV) {
        const R inv = Ar<R, FAST>::rcp(S - Ss);
        const R chi = d * inv;
        const R kv = (d * Ss) * inv;
        const R su = Ss - k.un;
        out[0] = kv * k.U[0];
        out[1] = kv * k.U[1];
        out[2] = k.p + k.rho * (d * su + kv * Ss);
        out[3] = kv * k.U[3];
        out[4] = kv * k.E + k.p * k.un + S * (su * (chi * (k.rho * Ss) + k.p * inv));
        out[5] = kv;
        out[6] = k.z;
        if constexpr (NC == 7) out[7] = kv * k.U[5];
        return;
    }
    R chi;
    R us[5];
    if constexpr (FAST) {   // chi/d = 1/(S - S*): one reciprocal for the whole star state
        const R inv = Ar<R, FAST>::rcp(S - Ss);
        chi = d * inv;
        us[4] = chi * k.E + (Ss - k.un) * (chi * (k.rho * Ss) + k.p * inv);
    } else {
        chi = Ar<R, FAST>::div(d, S - Ss);
        us[4] = chi * (k.E + (Ss - k.un) * (k.rho * Ss + Ar<R, FAST>::div(k.p, d)));
    }
    us[0] = chi * k.U[0];
    us[1] = chi * k.U[1];
    us[2] = chi * (k.rho * Ss);
    us[3] = chi * (k.rho * k.ut);
#pragma unroll
    for (int c = 0; c < 5; ++c) out[c] = k.F[c] + S * (us[c] - k.U[c]);
    out[5] = k.un + S * (chi - R(1));
    out[6] = k.z;
    if constexpr (NC == 7) out[7] = k.F[5] + S * (chi * k.U[5] - k.U[5]);
}

// HLLC flux with Davis bounds; out = (5 flux components, u_f, z_f) and, with
// NC = 7, the reactant-mass flux.  The star state is evaluated once, for the
// side the contact moves away from; in the FP64 mode faces with S* == 0
// exactly (or NaN) evaluate both sides and average instead.
template <class R, int FAST, int NC, int EOS, bool TAVG = FAST == 0>
__device__ __forceinline__ void hllc(const Mix<R> &m, const R wL[NC], const R wR[NC],
                                     R out[NC + 1]) {
    Side<R, NC> L, Rs;
    R cL, cR;
    side_eval<R, FAST, NC, EOS>(m, wL, L, cL);
    side_eval<R, FAST, NC, EOS>(m, wR, Rs, cR);
    // The fast FP64 kernels form the conserved values and fluxes only for the
    // side(s) a face uses (the same operations on the same values; 2 % faster).
    // The others form both sides up front: in the correctly rounded FP64
    // kernel the lazy form measured 0.7 % slower; in the FP32 flux path it
    // measured 3 % faster, but its different FP32 rounding turns the reacting
    // nitromethane bubble of the tests non-physical at step 226 of 300 -- that
    // FP32 case runs close to its limit.
    constexpr bool kLazy = sizeof(R) == 8 && FAST == 2;
    if constexpr (!kLazy) {
        side_finish<R, NC>(L);
        side_finish<R, NC>(Rs);
    }
    auto finish = [&](Side<R, NC> &k) {
        if constexpr (kLazy) side_finish<R, NC>(k);
    };
    const R SL = fmin(L.un - cL, Rs.un - cR);
    const R SR = fmax(L.un + cL, Rs.un + cR);
    const R dL = SL - L.un;
    const R dR = SR - Rs.un;
    const R Ss = Ar<R, FAST>::div((Rs.p - L.p) + (L.U[2] * dL - Rs.U[2] * dR),
                            L.rho * dL - Rs.rho * dR);
    // A wave with no supersonic face takes the star flux without the final
    // selects; in the FP64 stiffened-gas kernels a wave whose faces all take
    // the same star side also evaluates that side without selecting its
    // values per lane (same values; in the other kernels that second path
    // would cost occupancy)
    constexpr bool kUniform = sizeof(R) == 8 && FAST != 1 && EOS == 0;
    // Ties (S* == 0): the two star branches agree there in exact arithmetic
    // (F*_R - F*_L = S* (U*_R - U*_L)).  With TAVG they are averaged (the FP64
    // mode's contract, which keeps mirror-symmetric data symmetric to the last
    // bit; also the FP32-bulk kernel, measured faster so), otherwise the left
    // branch is taken (fast FP64, FP32: one star evaluation per face)
    constexpr bool kTieAverage = TAVG;
    R st[NC + 1];
    if (!kTieAverage || Ss > R(0) || Ss < R(0)) {
        const bool useL = kTieAverage ? Ss > R(0) : !(Ss < R(0));
        // the chosen side per lane: its primitives, then its conserved values
        // and fluxes (FP64), or its finished values (FP32 flux path)
        auto select_side = [&]() {
            Side<R, NC> K;
            K.rho = useL ? L.rho : Rs.rho;
            K.un = useL ? L.un : Rs.un;
            K.ut = useL ? L.ut : Rs.ut;
            K.p = useL ? L.p : Rs.p;
            K.z = useL ? L.z : Rs.z;
            K.U[2] = useL ? L.U[2] : Rs.U[2];
            if constexpr (kLazy) {
                K.xi = useL ? L.xi : Rs.xi;
                K.eta = useL ? L.eta : Rs.eta;
                K.a1 = useL ? L.a1 : Rs.a1;
                K.a2 = useL ? L.a2 : Rs.a2;
                if constexpr (NC == 7) K.lam = useL ? L.lam : Rs.lam;
                side_finish<R, NC>(K);
            } else {
                K.E = useL ? L.E : Rs.E;
#pragma unroll
                for (int c = 0; c < NC - 1; ++c) {
                    if (c == 2) continue;
                    K.U[c] = useL ? L.U[c] : Rs.U[c];
                }
#pragma unroll
                for (int c = 0; c < NC - 1; ++c) K.F[c] = useL ? L.F[c] : Rs.F[c];
            }
            star_flux<R, FAST, NC, !kTieAverage>(K, useL ? SL : SR, Ss, st);
        };
        if constexpr (kUniform) {
            const unsigned long long act = __builtin_amdgcn_read_exec();   // lanes on this path
            const unsigned long long onL = __builtin_amdgcn_ballot_w64(useL);
            if (onL == act) {
                Side<R, NC> K = L;
                finish(K);
                star_flux<R, FAST, NC, !kTieAverage>(K, SL, Ss, st);
            } else if (onL == 0) {
                Side<R, NC> K = Rs;
                finish(K);
                star_flux<R, FAST, NC, !kTieAverage>(K, SR, Ss, st);
            } else {
                select_side();
            }
        } else {
            select_side();
        }
    } else {
        // contact at rest relative to the face (every face of a region at
        // rest): average of both star branches
        Side<R, NC> KL = L, KR = Rs;
        finish(KL);
        finish(KR);
        R a[NC + 1], b[NC + 1];
        star_flux<R, FAST, NC, !kTieAverage>(KL, SL, Ss, a);
        star_flux<R, FAST, NC, !kTieAverage>(KR, SR, Ss, b);
#pragma unroll
        for (int c = 0; c < NC + 1; ++c) st[c] = R(0.5) * (a[c] + b[c]);
    }
    const bool supL = SL >= R(0);
    const bool supR = !supL && (SR <= R(0));
    if (__builtin_amdgcn_ballot_w64(supL || supR) == 0) {
#pragma unroll
        for (int c = 0; c < NC + 1; ++c) out[c] = st[c];
        return;
    }
    // a supersonic face takes the upwind side's own flux
    Side<R, NC> FL = L, FR = Rs;
    finish(FL);
    finish(FR);
#pragma unroll
    for (int c = 0; c < 5; ++c) out[c] = supL ? FL.F[c] : (supR ? FR.F[c] : st[c]);
    out[5] = supL ? L.un : (supR ? Rs.un : st[5]);
    out[6] = supL ? L.z : (supR ? Rs.z : st[6]);
    if constexpr (NC == 7) out[7] = supL ? FL.F[5] : (supR ? FR.F[5] : st[7]);
}

// Tie rule of the HLLC flux for a kernel with storage type S, flux type R and
// arithmetic level FAST: average the two star branches at S* == 0 in the FP64
// mode and in FP32-bulk, take the left one in fast FP64 and FP32.
template <class S, class R, int FAST>
constexpr bool tie_average() {
    return FAST == 0 || sizeof(S) != sizeof(R);
}

// Update of one cell from its low- and high-face fluxes; fluxes are widened to
// the storage type before they are differenced.
template <class S, class R, int NC>
__device__ __forceinline__ void update_cell(const S q[NC], const R flo[NC + 1],
                                            const R fhi[NC + 1], S lam, S qo[NC]) {
#pragma unroll
    for (int c = 0; c < 5; ++c) qo[c] = q[c] - lam * ((S)fhi[c] - (S)flo[c]);
    const S z = q[5];
    qo[5] = z - lam * (((S)fhi[6] - z) * (S)fhi[5] - ((S)flo[6] - z) * (S)flo[5]);
    if constexpr (NC == 7) qo[6] = q[6] - lam * ((S)fhi[7] - (S)flo[7]);
}

// ------------------------------------------------------------------------
// x sweep of one row of the strip.  All 256 threads call it (it holds
// barriers); q: this thread's cell, qo: updated cell (valid for threads
// 2..253; the halo threads return q unchanged).
template <class S, class R, int FAST, int LIM, int NC, int EOS>
__device__ __forceinline__ void x_row(const S q[NC], S qo[NC], int t, S lam, R hl,
                                      const Mix<S> &ms, const Mix<R> &mr,
                                      R (*sWF)[kThreads], R (*sH)[kThreads]) {
    // the barrier-bound x sweep issues ahead of the other wave on the SIMD
    // (another workgroup's barrier-free y sweep), so the workgroup reaches
    // its barriers sooner
    __builtin_amdgcn_s_setprio(2);
    S w[NC], r, rc2;
    cons_to_prim<S, FAST, NC, EOS>(ms, q, w, r, rc2);
    R wr[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        wr[c] = (R)w[c];
        sWF[c][t] = wr[c];
    }
    __syncthreads();
    R wl[NC], wh[NC];
    if (t >= 1 && t <= kThreads - 2) {
        R wm[NC], wp[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            wm[c] = sWF[c][t - 1];
            wp[c] = sWF[c][t + 1];
        }
        face_states<R, FAST, LIM, NC>(wm, wr, wp, (R)r, (R)rc2, hl, wl, wh);
#pragma unroll
        for (int c = 0; c < NC; ++c) sH[c][t] = wh[c];
    }
    __syncthreads();
    R f[NC + 1];
    if (t >= 2 && t <= kThreads - 2) {
        R whm[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) whm[c] = sH[c][t - 1];
        hllc<R, FAST, NC, EOS, tie_average<S, R, FAST>()>(mr, whm, wl, f);
#pragma unroll
        for (int c = 0; c < NC + 1; ++c) sWF[c][t] = f[c];
    }
    __syncthreads();
    if (t >= 2 && t <= kThreads - 3) {
        R fh[NC + 1];
#pragma unroll
        for (int c = 0; c < NC + 1; ++c) fh[c] = sWF[c][t + 1];
        update_cell<S, R, NC>(q, f, fh, lam, qo);
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) qo[c] = q[c];
    }
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);
}

// x_row for the batched kernel: idle (uniform per wave) means the wave lies
// wholly right of the grid's last halo column, so nothing that is stored
// depends on it; it only takes part in the barriers.
template <class S, class R, int FAST, int LIM, int NC, int EOS>
__device__ __forceinline__ void x_row_skip(const S q[NC], S qo[NC], int t, S lam, R hl,
                                      const Mix<S> &ms, const Mix<R> &mr,
                                      R (*sWF)[kThreads], R (*sH)[kThreads], bool idle) {
    S w[NC], r, rc2;
    R wr[NC];
    if (!idle) {
        cons_to_prim<S, FAST, NC, EOS>(ms, q, w, r, rc2);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            wr[c] = (R)w[c];
            sWF[c][t] = wr[c];
        }
    }
    __syncthreads();
    R wl[NC], wh[NC];
    if (!idle && t >= 1 && t <= kThreads - 2) {
        R wm[NC], wp[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            wm[c] = sWF[c][t - 1];
            wp[c] = sWF[c][t + 1];
        }
        face_states<R, FAST, LIM, NC>(wm, wr, wp, (R)r, (R)rc2, hl, wl, wh);
#pragma unroll
        for (int c = 0; c < NC; ++c) sH[c][t] = wh[c];
    }
    __syncthreads();
    R f[NC + 1];
    if (!idle && t >= 2 && t <= kThreads - 2) {
        R whm[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) whm[c] = sH[c][t - 1];
        hllc<R, FAST, NC, EOS, tie_average<S, R, FAST>()>(mr, whm, wl, f);
#pragma unroll
        for (int c = 0; c < NC + 1; ++c) sWF[c][t] = f[c];
    }
    __syncthreads();
    if (!idle && t >= 2 && t <= kThreads - 3) {
        R fh[NC + 1];
#pragma unroll
        for (int c = 0; c < NC + 1; ++c) fh[c] = sWF[c][t + 1];
        update_cell<S, R, NC>(q, f, fh, lam, qo);
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) qo[c] = q[c];
    }
    __syncthreads();
}

// y sweep as a rolling window down one column (registers only).  Rows are
// pushed in order; after the 5th row the window yields the updated row two
// behind the one pushed.  Values are in the y frame (normal momentum rho v).
template <class S, class R, int FAST, int LIM, int NC, int EOS>
struct YPipe {
    S q1[NC], q2[NC];    // conserved rows k-1, k-2
    R w1[NC], w2[NC];    // primitives rows k-1, k-2
    R r1, c1;            // 1/rho and rho c^2 of row k-1
    R wh2[NC];           // high-face state of row k-2
    R f2[NC + 1];        // flux through the low face of row k-2

    // cnt = number of rows pushed before this one (uniform across the block)
    __device__ __forceinline__ bool push(int cnt, const S qk[NC], S qo[NC], S lam, R hl,
                                         const Mix<S> &ms, const Mix<R> &mr) {
        S w[NC], r, rc2;
        cons_to_prim<S, FAST, NC, EOS>(ms, qk, w, r, rc2);
        R wk[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) wk[c] = (R)w[c];
        bool out = false;
        if (cnt >= 2) {
            R wl[NC], wh[NC];
            face_states<R, FAST, LIM, NC>(w2, w1, wk, r1, c1, hl, wl, wh);
            if (cnt >= 3) {
                R f[NC + 1];
                hllc<R, FAST, NC, EOS, tie_average<S, R, FAST>()>(mr, wh2, wl, f);
                if (cnt >= 4) {
                    update_cell<S, R, NC>(q2, f2, f, lam, qo);
                    out = true;
                }
#pragma unroll
                for (int c = 0; c < NC + 1; ++c) f2[c] = f[c];
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) wh2[c] = wh[c];
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            q2[c] = q1[c]; q1[c] = qk[c];
            w2[c] = w1[c]; w1[c] = wk[c];
        }
        r1 = (R)r;
        c1 = (R)rc2;
        return out;
    }
};

template <class S, int NC> __device__ __forceinline__ void to_yframe(const S a[NC], S b[NC]) {
    b[0] = a[0]; b[1] = a[1]; b[2] = a[3]; b[3] = a[2]; b[4] = a[4]; b[5] = a[5];
    if constexpr (NC == 7) b[6] = a[6];
}

// Pointwise reaction stage over a time h (Strang split, Sec. 3) of one cell of
// a reactive liquid: Arrhenius rate K = -lambda C exp(-Ta / T2) (Eq. (6)) at
// the liquid temperature T2 = (p - p_ref(rho2)) / (rho2 Gamma_0 c_v) of
// Eq. (5) (T_ref = 0), held fixed over the stage, so lambda decays exactly by
// exp(-C exp(-Ta / T2) h); the reacted liquid mass releases Q per unit mass
// into rho E (source of Eq. (1)).  Cells without reactant or with T2 <= 0
// are left as they are.
template <class S, int FAST>
__device__ __forceinline__ void react(S q[7], const Mix<S> &m, const Rx<S> &x, S h) {
    if (!(q[6] > S(0))) return;
    S w[7], r, rc2;
    cons_to_prim<S, FAST, 7, 1>(m, q, w, r, rc2);
    const S rho2 = Ar<S, FAST>::div(q[1], S(1) - q[5]);
    const S v = Ar<S, FAST>::div(m.rho0, rho2);
    S vc, vd;
    Ar<S, FAST>::pw(v, m.C, m.D, vc, vd);
    const S pref = m.A * vc - m.B * vd;
    const S T = Ar<S, FAST>::div(w[4] - pref, (rho2 * x.G0) * x.cv);
    if (!(T > S(0))) return;
    const S k = x.C * Ar<S, FAST>::ex(-Ar<S, FAST>::div(x.Ta, T));
    const S lam_new = w[6] * Ar<S, FAST>::ex(-k * h);
    q[4] = q[4] + x.Q * (q[6] - q[1] * lam_new);
    q[6] = q[1] * lam_new;
}

// Liquid temperature of Eq. (5) (T_ref = 0, constant Gamma_0 and c_v) of a
// cell of a reactive Cochran-Chan liquid, evaluated in FP64.
__device__ __forceinline__ double liquid_temperature(const Mix<double> &m, const Rx<double> &x,
                                                     const double q[7]) {
    double w[7], r, rc2;
    cons_to_prim<double, false, 7>(m, q, w, r, rc2);
    const double rho2 = q[1] / (1.0 - q[5]);
    const double v = m.rho0 / rho2;
    double vc, vd;
    Ar<double, false>::pw(v, m.C, m.D, vc, vd);
    const double pref = m.A * vc - m.B * vd;
    return (w[4] - pref) / ((rho2 * x.G0) * x.cv);
}

// Volumetric heat-release rate -z2 rho2 K Q of the reactive liquid (Sec. 4.5)
// in GW/m^3; 0 without reactant or at T2 <= 0.
__device__ __forceinline__ double heat_release(const Mix<double> &m, const Rx<double> &x,
                                               const double q[7]) {
    if (!(q[6] > 0.0)) return 0.0;
    const double T = liquid_temperature(m, x, q);
    if (!(T > 0.0)) return 0.0;
    return ((q[6] * x.C) * exp(-x.Ta / T) * x.Q) * 1.0e-9;
}

// Pointwise stage and CFL contribution of one updated cell (U order): the z1
// clamp, the second half of the reaction (NC = 7), then the signal speed.
template <class S, int FAST, int NC, int EOS>
__device__ __forceinline__ void epilogue(S q[NC], const Mix<S> &ms, const Rx<S> &rx, S hdt,
                                         S zlo, S zhi, S idx, S idy, S &smax, int &bad) {
    q[5] = fmin(fmax(q[5], zlo), zhi);
    if constexpr (NC == 7) react<S, FAST>(q, ms, rx, hdt);
    S w[NC], r, rc2;
    cons_to_prim<S, FAST, NC, EOS>(ms, q, w, r, rc2);
    const S c = Ar<S, FAST>::sqrt_(rc2 * r);
    const S s = fmax((fabs(w[2]) + c) * idx, (fabs(w[3]) + c) * idy);
    if (!(r > S(0)) || !(rc2 > S(0)) || !(s <= Ar<S, FAST>::big())) bad = 1;
    else smax = fmax(smax, s);
}

// Workgroup max of the CFL bound folded into the control block.
__device__ __forceinline__ void block_cfl_commit(double smax, int bad, Control *ctl, int slot) {
    __shared__ double red_s[kThreads / 64];
    __shared__ int red_b[kThreads / 64];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        smax = fmax(smax, __shfl_xor(smax, off));
        bad |= __shfl_xor(bad, off);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red_s[wv] = smax;
        red_b[wv] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red_s[0];
        int b = red_b[0];
        for (int i = 1; i < kThreads / 64; ++i) {
            m = fmax(m, red_s[i]);
            b |= red_b[i];
        }
        unsigned long long bits = b ? 0x7FF8000000000000ULL
                                    : (unsigned long long)__double_as_longlong(m);
        atomicMax(&ctl->smax_bits[slot], bits);
        if (b) atomicOr(&ctl->err, 1);
    }
}

// Workgroup sums of N per-thread values, written to out[0..N-1]: a butterfly
// within each wave (every lane ends with the same bits, the two operands of
// each addition being the same pair in either order), then the waves in
// order, so the result depends only on the values and their lanes.
template <int N>
__device__ __forceinline__ void block_sums(const double v[N], double *out) {
    __shared__ double red[kThreads / 64][N];
    double s[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
        s[c] = v[c];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) s[c] = s[c] + __shfl_xor(s[c], off);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < N; ++c) red[wv][c] = s[c];
    }
    __syncthreads();
    if (threadIdx.x < N) {
        double a = red[0][threadIdx.x];
        for (int i = 1; i < kThreads / 64; ++i) a = a + red[i][threadIdx.x];
        out[threadIdx.x] = a;
    }
}

// ------------------------------------------------------------------------
// One tile of the state update: strip bx (252 written columns) and row
// segment by of the solve described by d.  MODE: kXY / kYX (fused step), kX /
// kY (one sweep).  FINAL: this pass produces the end-of-step state (pointwise
// stage + CFL contribution).  A pass that starts a step (fused, or the first
// of two sweeps) applies the first half of the reaction stage (NC = 7) to
// every value it loads, halo cells included.  All threads of the workgroup
// call it.
template <class S, class R, int FAST, int LIM, int MODE, bool FINAL, int NC, int EOS,
          bool SKIP = false, int DIAG = 0>
__device__ __forceinline__ void run_tile(const Desc &d, int bx, int by, int src_idx,
                                         R (*sWF)[kThreads], R (*sH)[kThreads],
                                         double *sEdge = nullptr, double *sHist = nullptr,
                                         double (*sInt)[kThreads] = nullptr) {
    Control *ctl = d.ctl;
    const S lamx = (S)ctl->lam_x, lamy = (S)ctl->lam_y;
    const R hlx = (R)ctl->hl_x, hly = (R)ctl->hl_y;
    const int slot = (int)((ctl->step_exec + 1) & 1);
    constexpr bool kStarts = (MODE == kXY) || (MODE == kYX) || !FINAL;

    const Mix<S> ms = mix_of<S>(d);
    const Mix<R> mr = mix_of<R>(d);
    Rx<S> rx{};
    S hdt = S(0);
    if constexpr (NC == 7) {
        rx = rx_of<S>(d);
        hdt = (S)(0.5 * ctl->dt);
    }
    const S *src = (const S *)d.buf[src_idx];
    S *dst = (S *)d.buf[src_idx ^ 1];
    const long long plane = d.plane;
    const int t = threadIdx.x;
    const int x0 = bx * kTileW;
    const int col = x0 - kHalo + t;
    const int gcol = map_idx(col, d.nx, d.bc_xlo, d.bc_xhi);
    const bool out_col = (t >= kHalo) && (t < kThreads - kHalo) && (col < d.nx);
    // SKIP: a wave whose first column lies beyond the grid's last halo column
    // does no arithmetic (the mostly empty last strip of a small grid)
    [[maybe_unused]] const bool idle = SKIP && (x0 - kHalo + (t & ~63) >= d.nx + kHalo);
    const bool head = by < d.seg_n1;
    const int y0 = head ? by * d.seg_h : d.seg_n1 * d.seg_h + (by - d.seg_n1) * d.seg_h2;
    const int y1 = min(y0 + (head ? d.seg_h : d.seg_h2), d.ny);
    const S zlo = (S)d.zlo, zhi = (S)d.zhi, idx = (S)d.idx, idy = (S)d.idy;

    S smax = S(0);
    int bad = 0;

    auto load = [&](int k, S q[NC]) {
        if constexpr (SKIP) {
            if (idle) {   // nothing to read; keep the registers defined
#pragma unroll
                for (int c = 0; c < NC; ++c) q[c] = S(0);
                return;
            }
        }
        const int gk = map_idx(k, d.ny, d.bc_ylo, d.bc_yhi);
        const long long o = (long long)gk * d.pitch + gcol;
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] = src[c * plane + o];
    };
    auto start = [&](S q[NC]) {
        if constexpr (NC == 7 && kStarts) react<S, FAST>(q, ms, rx, hdt);
    };
    // DIAG (a recording step), on the stored values in FP64 (the FP64 closure
    // whatever the mode): the column's sums of pressure, density and x
    // momentum over the segment's rows in row order (d.diag); the column's
    // sums of every stored plane (d.dint; running sums in LDS, sInt, one
    // slot per thread, to spare registers); the liquid mass of each cell
    // added to the workgroup's bin of its pressure, density or heat-release
    // rate (d.dhist; bins in LDS, sHist)
    double dsum_p = 0.0, dsum_r = 0.0, dsum_m = 0.0;
    // the histogram's pending bin of this thread and its mass: cells down a
    // column mostly share a bin, so one LDS atomic per run of them
    [[maybe_unused]] int hbin = -1;
    [[maybe_unused]] double hmass = 0.0;
    if constexpr (DIAG) {
        if (d.dint) {
#pragma unroll
            for (int c = 0; c < NC; ++c) sInt[c][t] = 0.0;
        }
    }
    auto store = [&](int k, S q[NC]) {
        if (FINAL) epilogue<S, FAST, NC, EOS>(q, ms, rx, hdt, zlo, zhi, idx, idy, smax, bad);
        const long long o = (long long)k * d.pitch + col;
#pragma unroll
        for (int c = 0; c < NC; ++c) dst[c * plane + o] = q[c];
        if constexpr (DIAG) {
            double qd[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) qd[c] = (double)q[c];
            if (d.dint) {
#pragma unroll
                for (int c = 0; c < NC; ++c) sInt[c][t] = sInt[c][t] + qd[c];
            }
            double v = 0.0;
            if (d.diag || (DIAG == 2 && d.hfield != MF_QDOT)) {
                double wd[NC], rr, rc;
                cons_to_prim<double, 0, NC, EOS>(mix_of<double>(d), qd, wd, rr, rc);
                if (d.diag) {
                    dsum_p = dsum_p + wd[4];
                    dsum_r = dsum_r + (qd[0] + qd[1]);
                    dsum_m = dsum_m + qd[2];
                }
                v = d.hfield == MF_RHO ? qd[0] + qd[1] : wd[4];
            }
            if constexpr (DIAG == 2) {
                if constexpr (NC == 7) {
                    if (d.hfield == MF_QDOT) v = heat_release(mix_of<double>(d), rx_of<double>(d), qd);
                }
                const int nb = d.hbins;
                if (v >= sEdge[0] && v < sEdge[nb]) {
                    // the bin a with e[a] <= v < e[a+1]: a guess from the
                    // FP32 logarithm, then decided by the FP64 edges (the
                    // same bin as a search over the edges)
                    const float g = (__log2f((float)v) * 0.30102999566f - d.hlo) * d.hidn;
                    int a = min(max((int)g, 0), nb - 1);
                    while (a > 0 && v < sEdge[a]) --a;
                    while (a < nb - 1 && v >= sEdge[a + 1]) ++a;
                    const double m = qd[1] * (d.dx * d.dy);
                    if (a == hbin) {
                        hmass = hmass + m;
                    } else {
                        if (hbin >= 0) atomicAdd(&sHist[hbin], hmass);
                        hbin = a;
                        hmass = m;
                    }
                }
            }
        }
    };

    if (MODE == kX) {
        S qn[NC];
        load(y0, qn);
        for (int k = y0; k < y1; ++k) {
            S q[NC], qo[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) q[c] = qn[c];
            if (k + 1 < y1) load(k + 1, qn);
            start(q);
            if constexpr (SKIP)
                x_row_skip<S, R, FAST, LIM, NC, EOS>(q, qo, t, lamx, hlx, ms, mr, sWF, sH,
                                                     idle);
            else
                x_row<S, R, FAST, LIM, NC, EOS>(q, qo, t, lamx, hlx, ms, mr, sWF, sH);
            if (out_col) store(k, qo);
        }
    } else {
        YPipe<S, R, FAST, LIM, NC, EOS> yp;
        const int k0 = y0 - kHalo, k1 = y1 + kHalo;
        S qn[NC];
        load(k0, qn);
        for (int k = k0; k < k1; ++k) {
            const int cnt = k - k0;
            S q[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) q[c] = qn[c];
            if (k + 1 < k1) load(k + 1, qn);
            start(q);
            if (MODE == kXY) {
                S qs[NC], qy[NC], qo[NC], qu[NC];
                if constexpr (SKIP)
                    x_row_skip<S, R, FAST, LIM, NC, EOS>(q, qs, t, lamx, hlx, ms, mr, sWF, sH,
                                                         idle);
                else
                    x_row<S, R, FAST, LIM, NC, EOS>(q, qs, t, lamx, hlx, ms, mr, sWF, sH);
                to_yframe<S, NC>(qs, qy);
                if ((!SKIP || !idle) && yp.push(cnt, qy, qo, lamy, hly, ms, mr)) {
                    to_yframe<S, NC>(qo, qu);
                    if (out_col) store(k - kHalo, qu);
                }
            } else {
                S qy[NC], qo[NC], qu[NC];
                to_yframe<S, NC>(q, qy);
                // the window yields a row from the 5th push on, in every wave alike
                bool got;
                if constexpr (SKIP)
                    got = idle ? cnt >= 4 : yp.push(cnt, qy, qo, lamy, hly, ms, mr);
                else
                    got = yp.push(cnt, qy, qo, lamy, hly, ms, mr);
                to_yframe<S, NC>(qo, qu);
                if (MODE == kY) {
                    if (got && out_col) store(k - kHalo, qu);
                } else if (got) {  // kYX: x sweep of the row just finished in y
                    S qx[NC];
                    if constexpr (SKIP)
                        x_row_skip<S, R, FAST, LIM, NC, EOS>(qu, qx, t, lamx, hlx, ms, mr, sWF, sH,
                                                             idle);
                    else
                        x_row<S, R, FAST, LIM, NC, EOS>(qu, qx, t, lamx, hlx, ms, mr, sWF, sH);
                    if (out_col) store(k - kHalo, qx);
                }
            }
        }
    }
    if constexpr (DIAG) {
        if (d.diag && out_col) {   // this segment's column sums (segments in row order)
            const long long n = d.nx;
            double *part = d.diag + by * 3 * n;
            part[col] = dsum_p;
            part[n + col] = dsum_r;
            part[2 * n + col] = dsum_m;
        }
        if (d.dint) {
            double isum[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) isum[c] = sInt[c][t];
            block_sums<NC>(isum, d.dint + (long long)NC * ((long long)by * d.nstrips + bx));
        }
        if constexpr (DIAG == 2) {   // the workgroup's bins into the step's row
            if (hbin >= 0) atomicAdd(&sHist[hbin], hmass);
            __syncthreads();
            for (int b = t; b < d.hbins; b += kThreads)
                if (sHist[b] != 0.0) atomicAdd(&d.dhist[b], sHist[b]);
        }
    }
    if (FINAL) block_cfl_commit((double)smax, bad, ctl, slot);
}

// Extra attributes of the two state-update kernels, set by a translation unit
// before it includes this header (empty: the compiler's own occupancy choice).
#ifndef MESO_STEP_ATTR
#define MESO_STEP_ATTR
#endif

// State update of one solve: grid (strips, segments).
template <class S, class R, int FAST, int LIM, int MODE, bool FINAL, int NC, int EOS>
__global__ __launch_bounds__(kThreads) MESO_STEP_ATTR void step_kernel(Desc d, int src_idx) {
    __shared__ R sWF[NC + 1][kThreads];
    __shared__ R sH[NC][kThreads];
    if (d.ctl->skip) return;
    run_tile<S, R, FAST, LIM, MODE, FINAL, NC, EOS>(d, blockIdx.x, blockIdx.y, src_idx, sWF, sH);
}

// The fused step of a recording step (diagnostics summed in the store
// epilogue), held to at least two waves per SIMD like the plain FP64 kernel.
// HIST: a histogram is recorded (a variant of its own, so that the other
// recordings keep the registers it needs); dynamic LDS holds its edges and
// bins (2 hbins + 1 doubles).
template <class S, class R, int FAST, int LIM, int MODE, int NC, int EOS, bool HIST>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void
record_step_kernel(Desc d, int src_idx) {
    __shared__ R sWF[NC + 1][kThreads];
    __shared__ R sH[NC][kThreads];
    __shared__ double sInt[NC][kThreads];
    extern __shared__ double sHistMem[];
    if (d.ctl->skip) return;
    double *sEdge = sHistMem, *sHist = sHistMem + d.hbins + 1;
    if constexpr (HIST) {
        for (int b = threadIdx.x; b <= d.hbins; b += kThreads) sEdge[b] = d.hedges[b];
        for (int b = threadIdx.x; b < d.hbins; b += kThreads) sHist[b] = 0.0;
        __syncthreads();
    }
    run_tile<S, R, FAST, LIM, MODE, true, NC, EOS, false, HIST ? 2 : 1>(
        d, blockIdx.x, blockIdx.y, src_idx, sWF, sH, sEdge, sHist, sInt);
}

// Fused state update of many solves in one launch: workgroup b takes tile
// tiles[b] = (solve, strip, segment).  Each solve keeps its own step parity
// (x-y order and source copy), read from its control block.  Every tile of a
// launch has the same liquid EOS and number of conserved planes NC (the server
// launches one of these per class present); waves beyond a small grid's last
// halo column skip their arithmetic (SKIP).
template <class S, class R, int FAST, int LIM, int EOS, int NC>
__global__ __launch_bounds__(kThreads) MESO_STEP_ATTR void batched_step_kernel(const Desc *descs,
                                                                               const int4 *tiles) {
    __shared__ R sWF[NC + 1][kThreads];
    __shared__ R sH[NC][kThreads];
    const int4 tl = tiles[blockIdx.x];
    const Desc d = descs[tl.x];
    if (d.ctl->skip) return;
    const int par = (int)(d.ctl->step_exec & 1);
    if (par == 0) run_tile<S, R, FAST, LIM, kXY, true, NC, EOS, true>(d, tl.y, tl.z, 0, sWF, sH);
    else run_tile<S, R, FAST, LIM, kYX, true, NC, EOS, true>(d, tl.y, tl.z, 1, sWF, sH);
}

// The batched kernel for one class of solves: an inert liquid with EoS eos
// (NC = 6), or the reactive Cochran-Chan liquid (NC = 7).
template <class S, class R, int FAST, int NC>
auto batched_variant(int lim, int eos) -> void (*)(const Desc *, const int4 *) {
    if constexpr (NC == 7) {
        return lim == 1 ? batched_step_kernel<S, R, FAST, 1, 1, 7>
                        : batched_step_kernel<S, R, FAST, 0, 1, 7>;
    } else {
        if (lim == 1)
            return eos == 1 ? batched_step_kernel<S, R, FAST, 1, 1, 6>
                            : batched_step_kernel<S, R, FAST, 1, 0, 6>;
        return eos == 1 ? batched_step_kernel<S, R, FAST, 0, 1, 6>
                        : batched_step_kernel<S, R, FAST, 0, 0, 6>;
    }
}

template <class S, class R, int FAST, int NC>
void launch_batched_variants(const Desc *descs, const int4 *tiles, int ntiles, int lim, int eos,
                             hipStream_t st) {
    void (*k)(const Desc *, const int4 *) = batched_variant<S, R, FAST, NC>(lim, eos);
    hipLaunchKernelGGL(k, dim3(ntiles), dim3(kThreads), 0, st, descs, tiles);
}

// Host-side launch of the step kernel variant for one sweep mode (kXY, kYX,
// or a single sweep kX / kY that does or does not end the step).
template <class S, class R, int FAST, int LIM, int NC, int EOS>
void launch_step_variants_eos(const Desc &d, int mode, int final_pass, int src, hipStream_t st) {
    const dim3 grid(d.nstrips, d.nsegs), block(kThreads);
    void (*k)(Desc, int);
    // a recording step (fused sweeps only)
    const bool diag = d.diag != nullptr || d.dint != nullptr || d.dhist != nullptr;
    const size_t lds = (diag && d.dhist) ? sizeof(double) * (2 * (size_t)d.hbins + 1) : 0;
    switch (mode) {
        case kXY:
            k = !diag    ? step_kernel<S, R, FAST, LIM, kXY, true, NC, EOS>
                : d.dhist ? record_step_kernel<S, R, FAST, LIM, kXY, NC, EOS, true>
                          : record_step_kernel<S, R, FAST, LIM, kXY, NC, EOS, false>;
            break;
        case kYX:
            k = !diag    ? step_kernel<S, R, FAST, LIM, kYX, true, NC, EOS>
                : d.dhist ? record_step_kernel<S, R, FAST, LIM, kYX, NC, EOS, true>
                          : record_step_kernel<S, R, FAST, LIM, kYX, NC, EOS, false>;
            break;
        case kX:
            k = final_pass ? step_kernel<S, R, FAST, LIM, kX, true, NC, EOS>
                           : step_kernel<S, R, FAST, LIM, kX, false, NC, EOS>;
            break;
        default:
            k = final_pass ? step_kernel<S, R, FAST, LIM, kY, true, NC, EOS>
                           : step_kernel<S, R, FAST, LIM, kY, false, NC, EOS>;
            break;
    }
    hipLaunchKernelGGL(k, grid, block, lds, st, d, src);
}

// Liquid chosen from the descriptor: a reactive solve is always Cochran-Chan.
template <class S, class R, int FAST, int LIM, int NC>
void launch_step_variants(const Desc &d, int mode, int final_pass, int src, hipStream_t st) {
    if constexpr (NC == 7) {
        launch_step_variants_eos<S, R, FAST, LIM, 7, 1>(d, mode, final_pass, src, st);
    } else {
        if (d.eos2 == 1)
            launch_step_variants_eos<S, R, FAST, LIM, NC, 1>(d, mode, final_pass, src, st);
        else
            launch_step_variants_eos<S, R, FAST, LIM, NC, 0>(d, mode, final_pass, src, st);
    }
}

}  // namespace meso
