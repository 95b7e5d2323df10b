// collide.hpp -- node-local physics of the GPU library: moments, the
// Papanastasiou-regularised (PR) and implicitly-regularised (IR) collision of
// Regulski, Leonardi & Szumbarski (arXiv:1610.01388).
//
// All functions work on deviations h_i = f_i - w_i rho0 of the transformed
// populations (Sec. 2, Eq. 11), which keeps the small non-equilibrium
// moments accurate in reduced precision.  With Pi' = sum c c h the moments
// are rho = rho0 + sum h, j = sum c h, Pi = Pi' + rho0 cs^2 I.
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"

namespace lbm {

// PR: Papanastasiou-regularised with the explicit relaxation-time update
// (the strain rate uses the previous step's tau, kept per node); IR:
// implicitly regularised; PRI: PR with the implicit update of Sec. 3 (the
// tau consistent with its own strain rate, found per node; no state);
// IRHB: the IR construction for a Herschel-Bulkley fluid (K = nu_p, flow
// index n), its collision moment found per node (Sec. 3.2).
// OP_MRT is a flag on PR and PRI: MRT base collision (Sec. 2.1) instead of
// TRT, a separate kernel instantiation so that the TRT kernels do not carry
// its registers.  OP_FB, for FP32 / FP16 storage only, compiles in the FP64
// redo of near-yield nodes (without it the reduced-precision kernels carry
// no FP64 registers).
enum { OP_PR = 0, OP_IR = 1, OP_PRI = 2, OP_IRHB = 3, OP_MRT = 4, OP_FB = 8 };
__host__ __device__ constexpr int op_base(int op) { return op & 3; }
// TRT (or MRT) + EDM with a Papanastasiou viscosity
__host__ __device__ constexpr bool pr_family(int op) { return op_base(op) == OP_PR || op_base(op) == OP_PRI; }
// carries a relaxation-time field from step to step
__host__ __device__ constexpr bool has_tau(int op) { return op_base(op) == OP_PR; }
__host__ __device__ constexpr bool is_mrt(int op) { return (op & OP_MRT) != 0; }

__device__ __forceinline__ double d_sqrt(double v) { return sqrt(v); }
__device__ __forceinline__ float d_sqrt(float v) { return sqrtf(v); }
__device__ __forceinline__ double d_expm1(double v) { return expm1(v); }
__device__ __forceinline__ float d_expm1(float v) { return expm1f(v); }

// Per-launch constants in compute precision C.
template <class C> struct Coll {
    C rho0, nu_p, sigma_y, m, gamma_c, lambda, g[3];
    C sqrt2_sy;   // sqrt(2) sigma_y: IR yield threshold on |dev T|
    C ir_a, ir_b; // IR yielded: lambda = ir_a + ir_b / T, ir_a = (6nu_p-1)/(1+6nu_p),
                  // ir_b = 2 sqrt2 sigma_y/(1+6nu_p)  (Eqs. 39-40 combined)
    C pr_ec;      // PR: -expm1(-m gamma_c) / gamma_c  (nu_app at the cut-off is nu_p + sigma_y pr_ec / rho)
    C band;       // FP64 fallback band
    int axis;     // 0, or 1..3: known flow axis whose normal component the collision drops (Sec. 4.2.2)
    C mrt_b, mrt_e;  // MRT rates of the bulk moment and of the even moments of order >= 4 (<= 0: shear rate)
    C hb_n, hb_c;    // IRHB: flow index n and 3 K (3/sqrt 2)^(n-1)
};

template <class C> struct Moments {
    C drho, j[3];
    C p[6];  // Pi' = sum c c h: xx, yy, zz, xy, xz, yz
};

// Node state after the rheology solve, before relaxation.
template <class C> struct Pre {
    C rho, u[3];  // u: velocity inside the equilibrium (PR: j/rho; IR: j/rho + g/2)
    C a[6];       // IR: post-collision stress tensor A = lambda dev(T)
    C tau_p, tau_m, nu_app, gamma, Tn;
    bool unyielded, near_yield;
};

template <int LAT, class C>
__device__ __forceinline__ void add_c(C& acc, C v, int c)
{
    if (c == 1) acc += v;
    else if (c == -1) acc -= v;
}

// Eq. 9: zeroth, first and second moments (of the deviations).
// Accumulated in C from populations stored as H (the FP64 redo of a
// reduced-precision node sums its float values in double, no double copy).
// The velocities come in opposite pairs (i, i + 1 for odd i): the pair's sum
// carries the even moments (rho, Pi) and its difference the odd one (j), so
// each pair is combined once.
template <int LAT, class C, class H>
__device__ __forceinline__ Moments<C> moments_as(const H (&h)[Lattice<LAT>::Q])
{
    using L = Lattice<LAT>;
    Moments<C> mo;
    mo.drho = (C)h[0];
#pragma unroll
    for (int a = 0; a < 3; ++a) mo.j[a] = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a) mo.p[a] = 0;
#pragma unroll
    for (int i = 1; i < L::Q; i += 2) {
        const C hp = (C)h[i], hm = (C)h[i + 1];
        const C sum = hp + hm, dif = hp - hm;
        mo.drho += sum;
        add_c<LAT>(mo.j[0], dif, L::cx[i]);
        add_c<LAT>(mo.j[1], dif, L::cy[i]);
        add_c<LAT>(mo.j[2], dif, L::cz[i]);
        add_c<LAT>(mo.p[0], sum, L::cx[i] * L::cx[i]);
        add_c<LAT>(mo.p[1], sum, L::cy[i] * L::cy[i]);
        add_c<LAT>(mo.p[2], sum, L::cz[i] * L::cz[i]);
        add_c<LAT>(mo.p[3], sum, L::cx[i] * L::cy[i]);
        add_c<LAT>(mo.p[4], sum, L::cx[i] * L::cz[i]);
        add_c<LAT>(mo.p[5], sum, L::cy[i] * L::cz[i]);
    }
    return mo;
}

template <int LAT, class C>
__device__ __forceinline__ Moments<C> moments(const C (&h)[Lattice<LAT>::Q])
{
    return moments_as<LAT, C, C>(h);
}

// Non-equilibrium second moment Pi - rho cs^2 I - rho v v, from the
// deviation moments: Pi' - drho cs^2 I_d - rho v v.
template <int LAT, class C>
__device__ __forceinline__ void noneq_second(const Moments<C>& mo, C rho, const C (&v)[3], C (&t)[6])
{
    constexpr int D = Lattice<LAT>::D;
    const C third = C(1) / C(3);
    t[0] = mo.p[0] - mo.drho * third - rho * v[0] * v[0];
    t[1] = mo.p[1] - mo.drho * third - rho * v[1] * v[1];
    t[2] = (D == 3) ? mo.p[2] - mo.drho * third - rho * v[2] * v[2] : C(0);
    t[3] = mo.p[3] - rho * v[0] * v[1];
    t[4] = (D == 3) ? mo.p[4] - rho * v[0] * v[2] : C(0);
    t[5] = (D == 3) ? mo.p[5] - rho * v[1] * v[2] : C(0);
}

template <class C>
__device__ __forceinline__ C frob2(const C (&t)[6])
{
    return t[0] * t[0] + t[1] * t[1] + t[2] * t[2] + C(2) * (t[3] * t[3] + t[4] * t[4] + t[5] * t[5]);
}

// PRI: the relaxation time tau with tau = 1/2 + 3 nu_app(G / tau), G being
// the strain rate Eq. 24 gives at tau = 1.  F(tau) = tau - 1/2 - 3 nu_app(G /
// tau) is convex in tau and changes sign once on [1/2 + 3 nu_p, 1/2 + 3
// nu_0]; Newton's method, kept inside the shrinking bracket (bisection
// whenever a step would leave it), stops when a step is below the
// precision's resolution.  It starts at the root of the yielded asymptote
// when that lies in the bracket, else at the upper end.
template <class C>
__device__ __forceinline__ C implicit_tau(C G, const Coll<C>& p, C irho)
{
    const C s = p.sigma_y * irho;
    const C nu0 = p.nu_p + p.m * s;
    const C nuc = p.nu_p + s * p.pr_ec;
    C lo = C(0.5) + C(3) * p.nu_p;
    C hi = C(0.5) + C(3) * nu0;
    // Start: where the root lies once m gamma is large (yielded node,
    // nu_app ~ nu_p + s tau / G, linear in tau), else the upper end.
    const C r = C(3) * s;
    C x = hi;
    if (r < G) x = fmin(fmax(lo * G / (G - r), lo), hi);
    const C tol = sizeof(C) == 8 ? C(1e-14) : C(2e-7);
    for (int it = 0; it < 64; ++it) {
        const C gam = G / x;
        C nu, dnu;  // nu_app(gam) and d nu_app / d gam
        if (gam >= p.gamma_c) {
            const C em = -d_expm1(-p.m * gam);  // 1 - exp(-m gam)
            nu = p.nu_p + s * em / gam;
            dnu = s / gam * (p.m * (C(1) - em) - em / gam);
        } else {
            nu = nu0 + (gam / p.gamma_c) * (nuc - nu0);
            dnu = (nuc - nu0) / p.gamma_c;
        }
        const C F = x - C(0.5) - C(3) * nu;
        if (F > C(0)) hi = x;
        else lo = x;
        const C dF = C(1) + C(3) * dnu * G / (x * x);
        const C step = F / dF;
        C xn = x - step;
        // A step within tolerance ends the search before the bracket test:
        // at an exact root (F = 0) x has just become a bracket end, and the
        // strict test would send the next iterate off to the midpoint.
        const bool conv = fabs(step) <= tol * x;
        if (!conv && !(xn > lo && xn < hi)) xn = C(0.5) * (lo + hi);
        const bool done = conv || hi - lo <= tol * hi;
        x = xn;
        if (done) break;
    }
    return x;
}

__device__ __forceinline__ double d_pow(double b, double e) { return pow(b, e); }
__device__ __forceinline__ float d_pow(float b, float e) { return powf(b, e); }

// IRHB: magnitude s of the collision's second moment for a yielded node
// (Tn > sqrt(2) sigma_y).  The Herschel-Bulkley law written in s with the
// strain rate 3 s / sqrt(2) turns the contraction of Eq. 31 into
// F(s) = s/2 + c s^n + sqrt(2) sigma_y - Tn = 0, c = 3 K (3/sqrt 2)^(n-1):
// increasing in s and negative at 0; with e = Tn - sqrt(2) sigma_y the root
// lies below both 2 e (from s/2 <= e) and (e / c)^(1/n) (from c s^n <= e),
// the second bound close to it when the power term dominates (small n).
// Newton's method kept inside the shrinking bracket (bisection whenever a
// step would leave it) from the n = 1 closed form (exact for Bingham), until
// a step falls below the precision's resolution.  A bound that underflows
// to zero returns zero (s is then negligible against Tn).
template <class C>
__device__ __forceinline__ C hb_moment(C Tn, const Coll<C>& p)
{
    const C e = Tn - p.sqrt2_sy;
    C lo = C(0), hi = fmin(C(2) * e, d_pow(e / p.hb_c, C(1) / p.hb_n));
    if (!(hi > C(0))) return C(0);
    C x = fmin(e / (C(0.5) + p.hb_c), hi);
    const C tol = sizeof(C) == 8 ? C(1e-14) : C(2e-7);
    for (int it = 0; it < 64; ++it) {
        const C xn1 = d_pow(x, p.hb_n - C(1));  // s^(n-1); x > 0 here
        const C F = C(0.5) * x + p.hb_c * xn1 * x - e;
        if (F > C(0)) hi = x;
        else lo = x;
        const C step = F / (C(0.5) + p.hb_c * p.hb_n * xn1);
        C xn = x - step;
        const bool conv = fabs(step) <= tol * x;
        if (!conv && !(xn > lo && xn < hi)) xn = C(0.5) * (lo + hi);
        const bool done = conv || hi - lo <= tol * hi;
        x = xn;
        if (done) break;
    }
    return x;
}

// Rheology: everything up to, but not including, the relaxation.
//  PR (Sec. 2.2 Eq. 24, Sec. 3.1 Eqs. 36-37, Sec. 2.1): D from the
//   non-equilibrium second moment at the bare velocity with the previous
//   step's tau (density kept, as in Eq. 33), gamma = sqrt(2 D:D) on the full
//   tensor, nu_app with the linear interpolation below gamma_c (denominator
//   gamma_c), tau_even = 1/2 + 3 nu_app, tau_odd from Lambda.
//  PRI: as PR with tau_prev replaced by implicit_tau.
//  IR (Sec. 2.3, 3.2): T = sum c c (f - f_eq + Phi/2) at u = (j + F/2)/rho,
//   deviatoric part (trace / d), yielded iff |dev T| > sqrt(2) sigma_y,
//   A = -sigma + s/2 = lambda dev T with the closed forms of Eqs. 39-40.
template <int LAT, int OP, class C>
__device__ __forceinline__ Pre<C> rheology(const Moments<C>& mo, const Coll<C>& p, C tau_prev)
{
    constexpr int D = Lattice<LAT>::D;
    Pre<C> r;
    r.rho = p.rho0 + mo.drho;
    const C irho = C(1) / r.rho;
    if (pr_family(OP)) {
#pragma unroll
        for (int a = 0; a < 3; ++a) r.u[a] = mo.j[a] * irho;
        C t[6];
        noneq_second<LAT>(mo, r.rho, r.u, t);
        C tau_s = tau_prev;
        if (op_base(OP) == OP_PRI) {  // strain rate at tau = 1, then the self-consistent tau
            const C c1 = C(-1.5) * irho;
            C d1[6];
#pragma unroll
            for (int a = 0; a < 6; ++a) d1[a] = c1 * t[a];
            if (p.axis == 1) d1[0] = C(0);
            if (p.axis == 2) d1[1] = C(0);
            if (p.axis == 3) d1[2] = C(0);
            tau_s = implicit_tau(d_sqrt(C(2) * frob2(d1)), p, irho);
        }
        const C coef = C(-1.5) / (r.rho * tau_s);  // -1 / (2 rho cs^2 tau)
        C dd[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) dd[a] = coef * t[a];
        if (is_mrt(OP) && p.mrt_b > C(0)) {
            // Eq. 23 with MRT: the trace part relaxes at the bulk rate
            const C trd = ((D == 3) ? t[0] + t[1] + t[2] : t[0] + t[1]) / C(D);
            const C corr = C(-1.5) * irho * (p.mrt_b - C(1) / tau_s) * trd;
            dd[0] += corr;
            dd[1] += corr;
            if (D == 3) dd[2] += corr;
        }
        if (is_mrt(OP)) {
#pragma unroll
            for (int a = 0; a < 6; ++a) r.a[a] = t[a];  // non-equilibrium second moment
        }
        // known flow axis: its normal strain rate is a Burnett-order artefact
        if (p.axis == 1) dd[0] = C(0);
        if (p.axis == 2) dd[1] = C(0);
        if (p.axis == 3) dd[2] = C(0);
        const C gamma = d_sqrt(C(2) * frob2(dd));
        C nu;
        if (gamma >= p.gamma_c) {
            nu = p.nu_p + p.sigma_y * irho * (-d_expm1(-p.m * gamma)) / gamma;
        } else {
            const C nu0 = p.nu_p + p.m * p.sigma_y * irho;
            const C nuc = p.nu_p + p.sigma_y * irho * p.pr_ec;
            nu = nu0 + (gamma / p.gamma_c) * (nuc - nu0);
        }
        r.nu_app = nu;
        r.gamma = gamma;
        r.tau_p = C(0.5) + C(3) * nu;
        r.tau_m = C(0.5) + p.lambda / (r.tau_p - C(0.5));
        // the regularised stress magnitude sqrt(sigma:sigma / 2) = rho nu gamma
        // against the yield stress: unyielded below it, redone in FP64 (when
        // enabled) within the band around it
        const C stress = r.rho * nu * gamma;
        r.unyielded = stress < p.sigma_y;
        r.near_yield = p.sigma_y > C(0) && fabs(stress - p.sigma_y) < p.band * p.sigma_y;
        r.Tn = 0;
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) r.u[a] = mo.j[a] * irho + C(0.5) * p.g[a];
        C t[6];
        noneq_second<LAT>(mo, r.rho, r.u, t);
        // known flow axis: drop its normal component before the deviator
        if (p.axis == 1) t[0] = C(0);
        if (p.axis == 2) t[1] = C(0);
        if (p.axis == 3) t[2] = C(0);
        const C tr = (D == 3) ? t[0] + t[1] + t[2] : t[0] + t[1];
        const C trd = tr / C(D);
        t[0] -= trd;
        t[1] -= trd;
        if (D == 3) t[2] -= trd;
        const C Tn = d_sqrt(frob2(t));
        const bool yielded = Tn > p.sqrt2_sy;
        C lam = C(1);
        if (yielded) {
            if constexpr (op_base(OP) == OP_IRHB) lam = C(1) - hb_moment(Tn, p) / Tn;
            else lam = p.ir_a + p.ir_b / Tn;
        }
#pragma unroll
        for (int a = 0; a < 6; ++a) r.a[a] = lam * t[a];
        r.Tn = Tn;
        r.unyielded = !yielded;
        r.near_yield = p.sigma_y > C(0) && fabs(Tn - p.sqrt2_sy) < p.band * p.sqrt2_sy;
        r.tau_p = tau_prev;
        r.tau_m = tau_prev;
        r.nu_app = p.nu_p;
        r.gamma = 0;
    }
    return r;
}

// Relaxation: overwrite h with the post-collision deviations.
//  PR: TRT on the even/odd parts of h - h_eq, plus the EDM difference
//   f_eq(u + g) - f_eq(u) written out (Sec. 2.4, Eq. 34).
//  IR: f_eq(u) + f_sigma + Phi/2 with f_sigma = w/(2 cs^4)(c c - cs^2 I):A
//   and Phi = 3 w c.F, F = rho g (Sec. 2.3 Eqs. 28-29, Sec. 2.4 Eq. 35).
// Computed in C, read from and written to populations stored as H (H = C
// except in the FP64 redo of a reduced-precision node).
template <int LAT, int OP, class C, class H>
__device__ __forceinline__ void relax(H (&h)[Lattice<LAT>::Q], const Moments<C>& mo, const Pre<C>& r,
                                      const Coll<C>& p)
{
    using L = Lattice<LAT>;
    const C* u = r.u;
    const C uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    if (pr_family(OP)) {
        const C om_p = C(1) / r.tau_p;
        const C om_m = C(1) / r.tau_m;
        // MRT (Sec. 2.1): with the weights' inner product the second-order
        // Hermite projection of h - h_eq splits into shear (cc : Pi_dev) and
        // bulk ((tr/d)(|c|^2 - d cs^2)) parts; the remaining even moments take
        // om_e, the odd ones om_m:  even change = om_e n_s + (om_p - om_e) f2d
        // + (om_b - om_e) f2b.  Without MRT, om_e = om_b = om_p (TRT).
        constexpr bool mrt = is_mrt(OP);
        const C om_e = (mrt && p.mrt_e > C(0)) ? p.mrt_e : om_p;
        const C om_b = (mrt && p.mrt_b > C(0)) ? p.mrt_b : om_p;
        constexpr int D = L::D;
        const C* pn = r.a;
        const C trd = ((D == 3) ? pn[0] + pn[1] + pn[2] : pn[0] + pn[1]) / C(D);
        const C dsh = om_p - om_e, dbu = om_b - om_e;
        const C ug = p.g[0] * (C(2) * u[0] + p.g[0]) + p.g[1] * (C(2) * u[1] + p.g[1]) +
                     p.g[2] * (C(2) * u[2] + p.g[2]);
        {  // rest velocity: symmetric only (f2d = 0, f2b = -cs^2 d trd * 9/2 w = -1.5 w d trd)
            const C w = C(L::w[0]);
            const C es = w * (mo.drho - C(1.5) * r.rho * uu);
            const C h0 = (C)h[0];
            C ns0 = om_e * (h0 - es);
            if (mrt) ns0 += dbu * (C(-1.5) * w * C(D) * trd);
            h[0] = (H)(h0 - ns0 - C(1.5) * r.rho * w * ug);
        }
#pragma unroll
        for (int i = 1; i < L::Q; i += 2) {
            const int k = i + 1;
            const C w = C(L::w[i]);
            C cu = 0, cg = 0;
            add_c<LAT>(cu, u[0], L::cx[i]);
            add_c<LAT>(cu, u[1], L::cy[i]);
            add_c<LAT>(cu, u[2], L::cz[i]);
            add_c<LAT>(cg, p.g[0], L::cx[i]);
            add_c<LAT>(cg, p.g[1], L::cy[i]);
            add_c<LAT>(cg, p.g[2], L::cz[i]);
            const C es = w * (mo.drho + r.rho * (C(4.5) * cu * cu - C(1.5) * uu));
            const C ea = C(3) * w * r.rho * cu;
            const C hi = (C)h[i], hk = (C)h[k];
            const C hs = C(0.5) * (hi + hk);
            const C ha = C(0.5) * (hi - hk);
            C ns = om_e * (hs - es);
            if (mrt) {
                C cpc = 0;  // c c : Pi_neq
                add_c<LAT>(cpc, pn[0], L::cx[i] * L::cx[i]);
                add_c<LAT>(cpc, pn[1], L::cy[i] * L::cy[i]);
                add_c<LAT>(cpc, pn[2], L::cz[i] * L::cz[i]);
                add_c<LAT>(cpc, C(2) * pn[3], L::cx[i] * L::cy[i]);
                add_c<LAT>(cpc, C(2) * pn[4], L::cx[i] * L::cz[i]);
                add_c<LAT>(cpc, C(2) * pn[5], L::cy[i] * L::cz[i]);
                const int c2 = L::cx[i] * L::cx[i] + L::cy[i] * L::cy[i] + L::cz[i] * L::cz[i];
                const C f2d = C(4.5) * w * (cpc - trd * C(c2));
                const C f2b = C(4.5) * w * trd * (C(c2) - C(D) / C(3));
                ns += dsh * f2d + dbu * f2b;
            }
            const C na = om_m * (ha - ea);
            // f_eq(u+g) - f_eq(u) for +c and -c
            const C fs = r.rho * w * (C(4.5) * cg * (C(2) * cu + cg) - C(1.5) * ug);
            const C fa = r.rho * w * C(3) * cg;
            // the pair's post-collision symmetric and antisymmetric parts
            const C ps = hs - ns + fs, pa = ha - na + fa;
            h[i] = (H)(ps + pa);
            h[k] = (H)(ps - pa);
        }
    } else {
        // Per opposite pair (i, i + 1): the equilibrium's even part and the
        // stress term are shared, the odd part (velocity and force) changes
        // sign, so h_i = E + O and h_{i+1} = E - O.
        const C* A = r.a;
        const C trA = A[0] + A[1] + A[2];
        const C third = C(1) / C(3);
        const C trd = trA * third;
        const C even0 = mo.drho - C(1.5) * r.rho * uu;
        {
            const C w = C(L::w[0]);
            h[0] = (H)(w * even0 + C(4.5) * w * (C(0) - trd));
        }
        const C rho3 = C(3) * r.rho, rho15 = C(1.5) * r.rho, rho45 = C(4.5) * r.rho;
#pragma unroll
        for (int i = 1; i < L::Q; i += 2) {
            const C w = C(L::w[i]);
            C cu = 0, cg = 0;
            add_c<LAT>(cu, u[0], L::cx[i]);
            add_c<LAT>(cu, u[1], L::cy[i]);
            add_c<LAT>(cu, u[2], L::cz[i]);
            add_c<LAT>(cg, p.g[0], L::cx[i]);
            add_c<LAT>(cg, p.g[1], L::cy[i]);
            add_c<LAT>(cg, p.g[2], L::cz[i]);
            C cac = 0;
            add_c<LAT>(cac, A[0], L::cx[i] * L::cx[i]);
            add_c<LAT>(cac, A[1], L::cy[i] * L::cy[i]);
            add_c<LAT>(cac, A[2], L::cz[i] * L::cz[i]);
            add_c<LAT>(cac, C(2) * A[3], L::cx[i] * L::cy[i]);
            add_c<LAT>(cac, C(2) * A[4], L::cx[i] * L::cz[i]);
            add_c<LAT>(cac, C(2) * A[5], L::cy[i] * L::cz[i]);
            const C E = w * (even0 + rho45 * cu * cu) + C(4.5) * w * (cac - trd);
            const C O = w * (rho3 * cu + rho15 * cg);
            h[i] = (H)(E + O);
            h[i + 1] = (H)(E - O);
        }
    }
}

// Reported velocity j/rho + g/2 (both operators).
template <class C>
__device__ __forceinline__ void out_velocity(const Moments<C>& mo, const Pre<C>& r, const Coll<C>& p, C (&uo)[3])
{
    const C irho = C(1) / r.rho;
#pragma unroll
    for (int a = 0; a < 3; ++a) uo[a] = mo.j[a] * irho + C(0.5) * p.g[a];
}

}  // namespace lbm
