/*
 * lbm_oracle.c -- plain FP64 CPU reference of the lattice Boltzmann update for
 * Bingham fluids in Regulski, Leonardi & Szumbarski, "On the spatial
 * convergence and transient behaviour of lattice Boltzmann methods for
 * modelling fluids with yield stress" (arXiv:1610.01388).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark to check the GPU library.  It is deliberately
 * plain: one node at a time, every quantity computed from its definition, in
 * the order the paper introduces it, with no blocking, fusion or reordering.
 * Compiled without fast-math.
 *
 * Readings of passages that are garbled or silent in the paper are marked
 * "Reading:" where they are used.  All are pinned by tests (analytic flows,
 * conservation laws, the Newtonian limits).
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CS2 (1.0 / 3.0) /* lattice speed of sound squared, Sec. 2 */
#define QMAX 27

typedef struct {
    int d, q;
    int c[QMAX][3];
    double w[QMAX];
    int opp[QMAX];
    /* MRT moment basis (Sec. 2.1): row k of M is mrt[k][i], its weighted norm
     * sum_i w_i mrt[k][i]^2 is mrt_n[k], its rate group is mrt_group[k]. */
    double mrt[QMAX][QMAX];
    double mrt_n[QMAX];
    int mrt_group[QMAX];
} lattice_t;

enum { MRT_CONSERVED = 0, MRT_BULK = 1, MRT_SHEAR = 2, MRT_ODD = 3, MRT_EVEN = 4 };
static void build_mrt_basis(lattice_t* L);

/* The three velocity sets of Sec. 4.1.  The paper does not list them; these are
 * the standard sets: every c in {-1,0,1}^d, restricted to |c|^2 <= 2 for D3Q19,
 * with the standard weights for each speed class |c|^2.  The order is built
 * here by enumeration (z slowest, x fastest). */
static int build_lattice(int kind, lattice_t* L)
{
    double wk[4];
    int maxc2, dim;
    if (kind == ORC_D2Q9) {
        dim = 2; maxc2 = 2;
        wk[0] = 4.0 / 9.0; wk[1] = 1.0 / 9.0; wk[2] = 1.0 / 36.0; wk[3] = 0.0;
    } else if (kind == ORC_D3Q19) {
        dim = 3; maxc2 = 2;
        wk[0] = 1.0 / 3.0; wk[1] = 1.0 / 18.0; wk[2] = 1.0 / 36.0; wk[3] = 0.0;
    } else if (kind == ORC_D3Q27) {
        dim = 3; maxc2 = 3;
        wk[0] = 8.0 / 27.0; wk[1] = 2.0 / 27.0; wk[2] = 1.0 / 54.0; wk[3] = 1.0 / 216.0;
    } else {
        return -1;
    }
    L->d = dim;
    L->q = 0;
    int zlo = (dim == 3) ? -1 : 0, zhi = (dim == 3) ? 1 : 0;
    for (int cz = zlo; cz <= zhi; ++cz)
        for (int cy = -1; cy <= 1; ++cy)
            for (int cx = -1; cx <= 1; ++cx) {
                int c2 = cx * cx + cy * cy + cz * cz;
                if (c2 > maxc2) continue;
                L->c[L->q][0] = cx;
                L->c[L->q][1] = cy;
                L->c[L->q][2] = cz;
                L->w[L->q] = wk[c2];
                L->q++;
            }
    for (int i = 0; i < L->q; ++i) {
        L->opp[i] = -1;
        for (int k = 0; k < L->q; ++k)
            if (L->c[k][0] == -L->c[i][0] && L->c[k][1] == -L->c[i][1] &&
                L->c[k][2] == -L->c[i][2])
                L->opp[i] = k;
    }
    build_mrt_basis(L);
    return L->q;
}

/* MRT moment basis (Sec. 2.1, Eq. 20).  The paper names no basis; the one
 * used here is the Gram-Schmidt orthogonalisation, under the weighted inner
 * product <a, b> = sum_i w_i a_i b_i, of the monomials c_x^a c_y^b c_z^c
 * (a, b, c <= 2) taken in order of degree, with |c|^2 first among the
 * degree-2 ones; monomials that add nothing on the lattice are dropped.
 * Groups: degree 0-1 conserved, the |c|^2 row bulk, the other degree-2 rows
 * shear, odd degree >= 3 odd, even degree >= 4 even. */
static void build_mrt_basis(lattice_t* L)
{
    int nrow = 0;
    for (int deg = 0; deg <= 6; ++deg) {
        /* candidate monomials of this degree; at degree 2 the trace first */
        int cand[32][3], nc = 0;
        if (deg == 2) { cand[nc][0] = -1; nc++; }
        for (int a = 0; a <= 2; ++a)
            for (int b = 0; b <= 2; ++b)
                for (int cc = 0; cc <= 2; ++cc)
                    if (a + b + cc == deg) { cand[nc][0] = a; cand[nc][1] = b; cand[nc][2] = cc; nc++; }
        int first_deg2 = 1;
        for (int k = 0; k < nc; ++k) {
            double v[QMAX];
            for (int i = 0; i < L->q; ++i) {
                if (cand[k][0] < 0) {
                    v[i] = (double)(L->c[i][0] * L->c[i][0] + L->c[i][1] * L->c[i][1] + L->c[i][2] * L->c[i][2]);
                } else {
                    v[i] = 1.0;
                    for (int e = 0; e < cand[k][0]; ++e) v[i] *= L->c[i][0];
                    for (int e = 0; e < cand[k][1]; ++e) v[i] *= L->c[i][1];
                    for (int e = 0; e < cand[k][2]; ++e) v[i] *= L->c[i][2];
                }
            }
            double n0 = 0.0;
            for (int i = 0; i < L->q; ++i) n0 += L->w[i] * v[i] * v[i];
            for (int pass = 0; pass < 2; ++pass)
                for (int r = 0; r < nrow; ++r) {
                    double dot = 0.0;
                    for (int i = 0; i < L->q; ++i) dot += L->w[i] * v[i] * L->mrt[r][i];
                    for (int i = 0; i < L->q; ++i) v[i] -= dot / L->mrt_n[r] * L->mrt[r][i];
                }
            double n = 0.0;
            for (int i = 0; i < L->q; ++i) n += L->w[i] * v[i] * v[i];
            if (n <= 1e-12 * (n0 > 0.0 ? n0 : 1.0)) continue;
            for (int i = 0; i < L->q; ++i) L->mrt[nrow][i] = v[i];
            L->mrt_n[nrow] = n;
            if (deg <= 1) L->mrt_group[nrow] = MRT_CONSERVED;
            else if (deg == 2) { L->mrt_group[nrow] = first_deg2 ? MRT_BULK : MRT_SHEAR; first_deg2 = 0; }
            else L->mrt_group[nrow] = (deg % 2) ? MRT_ODD : MRT_EVEN;
            nrow++;
        }
    }
}

/* Omega = -M^{-1} S M (f - f_eq) (Eq. 20) with S from the group rates; with
 * rows orthogonal under the weights, M^{-1} = W M^T N^{-1}, so
 * (M^{-1} S M)_ij = sum_k s_k w_i m_k(i) m_k(j) / n_k. */
static void mrt_apply(const lattice_t* L, const double rate[5], const double* fneq, double* out)
{
    for (int i = 0; i < L->q; ++i) out[i] = 0.0;
    for (int k = 0; k < L->q; ++k) {
        double mk = 0.0;
        for (int j = 0; j < L->q; ++j) mk += L->mrt[k][j] * fneq[j];
        const double sk = rate[L->mrt_group[k]] * mk / L->mrt_n[k];
        for (int i = 0; i < L->q; ++i) out[i] += sk * L->w[i] * L->mrt[k][i];
    }
}

int orc_lattice_info(int lattice, int* d, int* c, double* w, int* opp)
{
    lattice_t L;
    if (build_lattice(lattice, &L) < 0) return -1;
    if (d) *d = L.d;
    for (int i = 0; i < L.q; ++i) {
        if (c) { c[3 * i] = L.c[i][0]; c[3 * i + 1] = L.c[i][1]; c[3 * i + 2] = L.c[i][2]; }
        if (w) w[i] = L.w[i];
        if (opp) opp[i] = L.opp[i];
    }
    return L.q;
}

/* ---------------------------------------------------------------------------
 * Node-local building blocks
 * ------------------------------------------------------------------------- */

/* Sec. 2.1, Eq. 12: second-order truncated Maxwell-Boltzmann equilibrium. */
static void equilibrium(const lattice_t* L, double rho, const double u[3], double* feq)
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < L->q; ++i) {
        double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
        feq[i] = rho * L->w[i] *
                 (1.0 + cu / CS2 + (cu * cu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

int orc_equilibrium(int lattice, double rho, const double* u, double* feq)
{
    lattice_t L;
    if (build_lattice(lattice, &L) < 0) return -1;
    equilibrium(&L, rho, u, feq);
    return L.q;
}

/* Sec. 2, Eq. 9: zeroth and first moments. */
static void density_momentum(const lattice_t* L, const double* f, double* rho, double j[3])
{
    *rho = 0.0;
    j[0] = j[1] = j[2] = 0.0;
    for (int i = 0; i < L->q; ++i) {
        *rho += f[i];
        for (int a = 0; a < 3; ++a) j[a] += L->c[i][a] * f[i];
    }
}

/* Second moment of a difference of two population sets: sum_i c_i c_i (f - h). */
static void second_moment_of_difference(const lattice_t* L, const double* f,
                                        const double* h, double M[3][3])
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[a][b] = 0.0;
    for (int i = 0; i < L->q; ++i) {
        double df = f[i] - h[i];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) M[a][b] += L->c[i][a] * L->c[i][b] * df;
    }
}

/* Sec. 3.1, Eq. 36 with the zero-strain interpolation of Eq. 37.
 * Reading: Eq. 37 as printed divides its first term by gamma_dot; the
 * interpolation it describes (linear between nu_0 at zero strain and
 * nu_app(gamma_c) at the cut-off, continuous at both ends) has gamma_c in that
 * denominator.  It is written here as nu_0 + (gamma/gamma_c)(nu_c - nu_0),
 * the same straight line, which returns nu_p exactly when sigma_y = 0.
 * 1 - exp(-m gamma) is evaluated as -expm1(-m gamma). */
double orc_nu_app(const orc_rheology* rh, double gamma, double rho)
{
    if (gamma >= rh->gamma_c)
        return rh->nu_p + rh->sigma_y / (rho * gamma) * (-expm1(-rh->m * gamma));
    double nu0 = rh->nu_p + rh->m * rh->sigma_y / rho;
    double nuc = rh->nu_p + rh->sigma_y / (rho * rh->gamma_c) * (-expm1(-rh->m * rh->gamma_c));
    return nu0 + (gamma / rh->gamma_c) * (nuc - nu0);
}

/* ---------------------------------------------------------------------------
 * PR: Papanastasiou-regularised model with explicit relaxation-time update
 * (Sec. 3, 3.1), TRT collision (Sec. 2.1) and EDM body force (Sec. 2.4).
 * ------------------------------------------------------------------------- */
static void collide_pr(const lattice_t* L, const orc_rheology* rh, const double* fbar,
                       double tau_prev, double* fpost, double* out)
{
    double rho, j[3], u[3], feq[QMAX], feq_shift[QMAX], ushift[3];
    double Pneq[3][3], D[3][3];

    /* Moments (Eq. 9).  Reading: the equilibrium that the TRT relaxes towards
     * and that defines the non-equilibrium part is the one at the bare
     * velocity j/rho; the force enters only through the EDM difference
     * (Eq. 34), and u + du/2 is the reported flow velocity. */
    density_momentum(L, fbar, &rho, j);
    for (int a = 0; a < 3; ++a) u[a] = j[a] / rho;
    equilibrium(L, rho, u, feq);

    /* Strain rate from the non-equilibrium second moment (Sec. 2.2, Eq. 24),
     * using the relaxation time of the previous step (explicit update,
     * Sec. 3).  Reading: Eq. 24 omits the density that Eq. 33 carries; the
     * density is kept (D = -Pi_neq / (2 rho cs^2 tau)). */
    const int mrt = rh->mrt_bulk > 0.0 || rh->mrt_even > 0.0;
    double fneq[QMAX];
    for (int i = 0; i < L->q; ++i) fneq[i] = fbar[i] - feq[i];
    if (!mrt) {
        second_moment_of_difference(L, fbar, feq, Pneq);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) D[a][b] = -Pneq[a][b] / (2.0 * rho * CS2 * tau_prev);
    } else {
        /* Eq. 23: D from the second moment of M^{-1} S M (f - f_eq), with the
         * shear rate of the previous step and the bulk rate as given. */
        double rate[5] = {0.0, rh->mrt_bulk > 0.0 ? rh->mrt_bulk : 1.0 / tau_prev, 1.0 / tau_prev, 0.0, 0.0};
        double g[QMAX];
        mrt_apply(L, rate, fneq, g);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double s2 = 0.0;
                for (int i = 0; i < L->q; ++i) s2 += L->c[i][a] * L->c[i][b] * g[i];
                D[a][b] = -s2 / (2.0 * rho * CS2);
            }
    }

    /* Sec. 4.2.2: for a flow known to run along one axis, the normal
     * component of the strain rate along it (a Burnett-order artefact of the
     * kinetic stress) can be set to zero. */
    if (rh->flow_axis >= 1 && rh->flow_axis <= 3) D[rh->flow_axis - 1][rh->flow_axis - 1] = 0.0;

    /* Characteristic strain rate (Sec. 1, Eq. 4), full tensor. */
    double DD = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) DD += D[a][b] * D[a][b];
    double gamma = sqrt(2.0 * DD);

    /* Apparent viscosity (Eqs. 36-37) and the relaxation times: tau from
     * nu = cs^2 (tau - 1/2) (Eq. 15) for the even modes; the odd-mode time
     * from the magic number Lambda = (tau_even - 1/2)(tau_odd - 1/2). */
    double nu_app = orc_nu_app(rh, gamma, rho);
    double tau_even = 0.5 + nu_app / CS2;
    double tau_odd = 0.5 + rh->lambda / (tau_even - 0.5);

    /* EDM (Eq. 34): add f_eq(u + du) - f_eq(u), du = F dt / rho = g. */
    for (int a = 0; a < 3; ++a) ushift[a] = u[a] + rh->g[a];
    equilibrium(L, rho, ushift, feq_shift);

    if (!mrt) {
        /* TRT: symmetric and antisymmetric parts under i <-> opposite(i). */
        for (int i = 0; i < L->q; ++i) {
            int k = L->opp[i];
            double f_sym = 0.5 * (fbar[i] + fbar[k]);
            double f_asym = 0.5 * (fbar[i] - fbar[k]);
            double e_sym = 0.5 * (feq[i] + feq[k]);
            double e_asym = 0.5 * (feq[i] - feq[k]);
            double omega = -(f_sym - e_sym) / tau_even - (f_asym - e_asym) / tau_odd;
            fpost[i] = fbar[i] + omega + (feq_shift[i] - feq[i]);
        }
    } else {
        /* MRT (Eq. 20): shear moments at 1/tau_even, odd moments at
         * 1/tau_odd (the magic number), bulk and higher even moments at
         * their own rates. */
        double rate[5] = {0.0, rh->mrt_bulk > 0.0 ? rh->mrt_bulk : 1.0 / tau_even, 1.0 / tau_even,
                          1.0 / tau_odd, rh->mrt_even > 0.0 ? rh->mrt_even : 1.0 / tau_even};
        double om[QMAX];
        mrt_apply(L, rate, fneq, om);
        for (int i = 0; i < L->q; ++i) fpost[i] = fbar[i] - om[i] + (feq_shift[i] - feq[i]);
    }

    /* Stress magnitude sqrt(sigma:sigma/2) = rho nu_app gamma for
     * sigma = 2 rho nu_app D; below sigma_y the node counts as unyielded
     * (Sec. 1, Eq. 1). */
    double stress = rho * nu_app * gamma;
    if (out) {
        out[0] = tau_even;
        out[1] = nu_app;
        out[2] = gamma;
        for (int a = 0; a < 3; ++a) out[3 + a] = u[a] + 0.5 * rh->g[a];
        out[6] = (stress < rh->sigma_y) ? 1.0 : 0.0;
    }
}

/* ---------------------------------------------------------------------------
 * IR: implicitly-regularised model (Sec. 2.3 and 3.2) with its own body
 * force term (Sec. 2.4, Eq. 35).
 * ------------------------------------------------------------------------- */
/* Herschel-Bulkley law written in s, in the manner of Eq. 38.  With a
 * Newtonian law Eqs. 32-33 identify D = 3 s / 2 (per unit density), so the
 * strain rate is g = sqrt(2 D:D) = 3 |s| / sqrt(2).  The law
 * sigma = 2 nu_app(g) D with nu_app = K g^(n-1) + sigma_y / g then reads
 * sigma = (3 K (3|s|/sqrt 2)^(n-1) + sqrt(2) sigma_y / |s|) s, which is
 * Eq. 38 for n = 1, K = nu_p.  With s and sigma along -T (as in the
 * Bingham case) the contraction of Eq. 31 leaves one equation for |s|:
 * F(s) = s/2 + 3 K (3/sqrt 2)^(n-1) s^n + sqrt(2) sigma_y - |T| = 0.
 * F increases with s, is negative at s = 0 when |T| > sqrt(2) sigma_y and
 * positive at s = 2 (|T| - sqrt(2) sigma_y): bisection to adjacent doubles. */
static double hb_F(const orc_rheology* rh, double s, double Tn)
{
    const double c = 3.0 * rh->nu_p * pow(3.0 / sqrt(2.0), rh->hb_n - 1.0);
    return 0.5 * s + c * pow(s, rh->hb_n) + sqrt(2.0) * rh->sigma_y - Tn;
}

static double hb_root(const orc_rheology* rh, double Tn)
{
    double lo = 0.0, hi = 2.0 * (Tn - sqrt(2.0) * rh->sigma_y);
    for (int it = 0; it < 4000; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (hb_F(rh, mid, Tn) > 0.0) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

static void collide_ir(const lattice_t* L, const orc_rheology* rh, const double* fbar,
                       double* fpost, double* out)
{
    double rho, j[3], u[3], F[3], feq[QMAX], phi[QMAX], feq_back[QMAX];
    double T[3][3], Tdev[3][3], s[3][3], sig[3][3], A[3][3];
    const double sqrt2 = sqrt(2.0);

    density_momentum(L, fbar, &rho, j);
    for (int a = 0; a < 3; ++a) F[a] = rho * rh->g[a];

    /* Reading: f_eq is taken half a time step back, i.e. Phi/2 is subtracted
     * from Eq. 12.  The velocity inside f_eq is (j + F/2)/rho so that the
     * post-collision momentum is j + F. */
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * F[a]) / rho;
    equilibrium(L, rho, u, feq);

    /* Force term (Eq. 35).  Reading: the printed coefficient 4 w_i (c.F)/rho
     * does not put momentum F into the fluid; the term with
     * sum_i c_i Phi_i = F is Phi_i = w_i (c_i . F) / cs^2 = 3 w_i c_i . F. */
    for (int i = 0; i < L->q; ++i) {
        double cF = L->c[i][0] * F[0] + L->c[i][1] * F[1] + L->c[i][2] * F[2];
        phi[i] = L->w[i] * cF / CS2;
        feq_back[i] = feq[i] - 0.5 * phi[i];
    }

    /* T = sum c c (fbar - f_eq) (Sec. 2.3, below Eq. 31). */
    second_moment_of_difference(L, fbar, feq_back, T);

    /* Sec. 4.2.2: with the flow direction known, T's normal component along
     * it is set to zero before the deviator, so it is not redistributed to
     * the transverse directions. */
    if (rh->flow_axis >= 1 && rh->flow_axis <= 3) T[rh->flow_axis - 1][rh->flow_axis - 1] = 0.0;

    /* Reading: only the deviatoric part enters (text below Eq. 29); the
     * printed sigma - Tr(sigma) I is read as sigma - Tr(sigma)/d I, applied
     * to T before the solve so that s and sigma are deviatoric. */
    double tr = 0.0;
    for (int a = 0; a < L->d; ++a) tr += T[a][a];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            Tdev[a][b] = T[a][b] - ((a == b && a < L->d) ? tr / L->d : 0.0);
    double TT = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) TT += Tdev[a][b] * Tdev[a][b];
    double Tn = sqrt(TT);

    /* Solve s/2 + T = -sigma (Eq. 31) with the Bingham law written in s
     * (Eq. 38): closed forms of Eqs. 39-40.  Reading: the yield test printed
     * as T >= sigma_y is T > sqrt(2) sigma_y -- the value at which the
     * yielded branch gives s = 0, so both branches meet there.  IRHB: the
     * same equation for a Herschel-Bulkley fluid, solved numerically. */
    int unyielded;
    if (Tn > sqrt2 * rh->sigma_y) {
        double s_mag, sig_mag;
        if (rh->op == ORC_IRHB) {
            s_mag = hb_root(rh, Tn);
            sig_mag = Tn - 0.5 * s_mag;  /* contraction of Eq. 31 with s, sigma along -T */
        } else {
            s_mag = (Tn - sqrt2 * rh->sigma_y) / (0.5 + 3.0 * rh->nu_p);
            sig_mag = (6.0 * rh->nu_p * Tn + sqrt2 * rh->sigma_y) / (1.0 + 6.0 * rh->nu_p);
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                s[a][b] = -s_mag * Tdev[a][b] / Tn;
                sig[a][b] = -sig_mag * Tdev[a][b] / Tn;
            }
        unyielded = 0;
    } else {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                s[a][b] = 0.0;
                sig[a][b] = -Tdev[a][b];
            }
        unyielded = 1;
    }

    /* f_sigma carries -sigma + s/2 (Eq. 29).  Reading: the printed prefactor
     * 3/2 w_i does not give f_sigma the second moment -sigma + s/2 that the
     * construction requires (nor the BGK limit of Eqs. 32-33); the Hermite
     * form w_i/(2 cs^4) (c_i c_i - cs^2 I) : A does. */
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) A[a][b] = -sig[a][b] + 0.5 * s[a][b];
    for (int i = 0; i < L->q; ++i) {
        double contr = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double H = L->c[i][a] * L->c[i][b] - ((a == b && a < L->d) ? CS2 : 0.0);
                contr += H * A[a][b];
            }
        double f_sigma = L->w[i] / (2.0 * CS2 * CS2) * contr;
        /* Eq. 28: post-collision = f_eq (half step back) + f_sigma + Phi. */
        fpost[i] = feq_back[i] + f_sigma + phi[i];
    }

    if (out) {
        for (int a = 0; a < 3; ++a) out[a] = u[a];
        out[3] = Tn;
        out[4] = unyielded;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                out[5 + 3 * a + b] = s[a][b];
                out[14 + 3 * a + b] = sig[a][b];
            }
    }
}

/* ---------------------------------------------------------------------------
 * Newtonian reference: BGK (Sec. 2.1, Eq. 14) with the EDM force (Eq. 34).
 * ------------------------------------------------------------------------- */
static void collide_bgk(const lattice_t* L, const orc_rheology* rh, const double* fbar,
                        double* fpost, double* out)
{
    double rho, j[3], u[3], feq[QMAX], feq_shift[QMAX], ushift[3];
    density_momentum(L, fbar, &rho, j);
    for (int a = 0; a < 3; ++a) u[a] = j[a] / rho;
    equilibrium(L, rho, u, feq);
    for (int a = 0; a < 3; ++a) ushift[a] = u[a] + rh->g[a];
    equilibrium(L, rho, ushift, feq_shift);
    double tau = 0.5 + rh->nu_p / CS2;
    for (int i = 0; i < L->q; ++i)
        fpost[i] = fbar[i] - (fbar[i] - feq[i]) / tau + (feq_shift[i] - feq[i]);
    if (out)
        for (int a = 0; a < 3; ++a) out[a] = u[a] + 0.5 * rh->g[a];
}

/* ---------------------------------------------------------------------------
 * PR with the implicit relaxation-time update (Sec. 3): instead of taking
 * the strain rate with the previous step's relaxation time, the collision
 * uses the relaxation time tau that reproduces itself: the strain rate of
 * Eq. 24 evaluated with tau gives, through Eqs. 36-37 and Eq. 15,
 * tau = 1/2 + nu_app / cs^2 again.  With G the strain rate Eq. 24 gives for
 * tau = 1, the strain rate at tau is G / tau, so tau is a root of
 *   F(tau) = tau - 1/2 - nu_app(G / tau) / cs^2,
 * which lies in [1/2 + nu_p / cs^2, 1/2 + nu_0 / cs^2] (nu_p <= nu_app <= nu_0)
 * where F changes sign.  It is found by bisection to the last bit, and the
 * collision is then the PR collision with that tau in place of the
 * previous one.
 * ------------------------------------------------------------------------- */
static double strain_rate_unit_tau(const lattice_t* L, const orc_rheology* rh, const double* fbar)
{
    double rho, j[3], u[3], feq[QMAX], Pneq[3][3], D[3][3];
    density_momentum(L, fbar, &rho, j);
    for (int a = 0; a < 3; ++a) u[a] = j[a] / rho;
    equilibrium(L, rho, u, feq);
    second_moment_of_difference(L, fbar, feq, Pneq);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) D[a][b] = -Pneq[a][b] / (2.0 * rho * CS2);
    if (rh->flow_axis >= 1 && rh->flow_axis <= 3) D[rh->flow_axis - 1][rh->flow_axis - 1] = 0.0;
    double DD = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) DD += D[a][b] * D[a][b];
    return sqrt(2.0 * DD);
}

static void collide_pri(const lattice_t* L, const orc_rheology* rh, const double* fbar,
                        double* fpost, double* out)
{
    double rho = 0.0;
    for (int i = 0; i < L->q; ++i) rho += fbar[i];
    const double G = strain_rate_unit_tau(L, rh, fbar);
    double lo = 0.5 + rh->nu_p / CS2;
    double hi = 0.5 + (rh->nu_p + rh->m * rh->sigma_y / rho) / CS2;
    for (int it = 0; it < 4000; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;  /* bracket is down to adjacent doubles */
        const double F = mid - 0.5 - orc_nu_app(rh, G / mid, rho) / CS2;
        if (F > 0.0) hi = mid;
        else lo = mid;
    }
    collide_pr(L, rh, fbar, 0.5 * (lo + hi), fpost, out);
}

int orc_collide_pri(int lattice, const orc_rheology* rh, const double* fbar,
                    double* fpost, double* out)
{
    lattice_t L;
    if (build_lattice(lattice, &L) < 0) return -1;
    collide_pri(&L, rh, fbar, fpost, out);
    return 0;
}

int orc_collide_pr(int lattice, const orc_rheology* rh, const double* fbar,
                   double tau_prev, double* fpost, double* out)
{
    lattice_t L;
    if (build_lattice(lattice, &L) < 0) return -1;
    collide_pr(&L, rh, fbar, tau_prev, fpost, out);
    return 0;
}

int orc_collide_ir(int lattice, const orc_rheology* rh, const double* fbar,
                   double* fpost, double* out)
{
    lattice_t L;
    if (build_lattice(lattice, &L) < 0) return -1;
    collide_ir(&L, rh, fbar, fpost, out);
    return 0;
}

int orc_collide_bgk(int lattice, const orc_rheology* rh, const double* fbar,
                    double* fpost, double* out)
{
    lattice_t L;
    if (build_lattice(lattice, &L) < 0) return -1;
    collide_bgk(&L, rh, fbar, fpost, out);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Domain: streaming with periodic wrap and halfway bounce-back.
 * ------------------------------------------------------------------------- */
struct orc_domain {
    lattice_t L;
    int n[3];
    int periodic[3];
    int64_t N;
    uint8_t* solid;  /* N */
    double* P;       /* q*N post-collision populations of the last step */
    double* Pnew;    /* q*N */
    double* tau;     /* N, PR relaxation time of the last step */
    double* taunew;  /* N */
    orc_rheology rh;
    int64_t t;
};

orc_domain* orc_create(int lattice, int nx, int ny, int nz, const int* periodic,
                       const uint8_t* mask, const orc_rheology* rh)
{
    orc_domain* dom = (orc_domain*)calloc(1, sizeof(orc_domain));
    if (!dom) return NULL;
    if (build_lattice(lattice, &dom->L) < 0 || nx < 1 || ny < 1 || nz < 1 ||
        (dom->L.d == 2 && nz != 1)) {
        free(dom);
        return NULL;
    }
    dom->n[0] = nx; dom->n[1] = ny; dom->n[2] = nz;
    for (int a = 0; a < 3; ++a) dom->periodic[a] = periodic ? periodic[a] : 1;
    if (dom->L.d == 2) dom->periodic[2] = 1; /* no z neighbours in 2-D */
    dom->N = (int64_t)nx * ny * nz;
    dom->rh = *rh;
    dom->solid = (uint8_t*)calloc((size_t)dom->N, 1);
    dom->P = (double*)calloc((size_t)(dom->L.q * dom->N), sizeof(double));
    dom->Pnew = (double*)calloc((size_t)(dom->L.q * dom->N), sizeof(double));
    dom->tau = (double*)calloc((size_t)dom->N, sizeof(double));
    dom->taunew = (double*)calloc((size_t)dom->N, sizeof(double));
    if (!dom->solid || !dom->P || !dom->Pnew || !dom->tau || !dom->taunew) {
        orc_destroy(dom);
        return NULL;
    }
    if (mask) memcpy(dom->solid, mask, (size_t)dom->N);
    orc_init_equilibrium(dom, 1.0, NULL);
    return dom;
}

void orc_destroy(orc_domain* dom)
{
    if (!dom) return;
    free(dom->solid); free(dom->P); free(dom->Pnew); free(dom->tau); free(dom->taunew);
    free(dom);
}

int64_t orc_time(const orc_domain* dom) { return dom->t; }

/* Start from rest (Sec. 4.4: an impulsively started, quiescent fluid). */
void orc_init_equilibrium(orc_domain* dom, double rho0, const double* u0)
{
    double u[3] = {0.0, 0.0, 0.0}, feq[QMAX];
    if (u0) { u[0] = u0[0]; u[1] = u0[1]; u[2] = u0[2]; }
    equilibrium(&dom->L, rho0, u, feq);
    double nu0 = dom->rh.nu_p + dom->rh.m * dom->rh.sigma_y / rho0;
    for (int64_t n = 0; n < dom->N; ++n) {
        for (int i = 0; i < dom->L.q; ++i)
            dom->P[i * dom->N + n] = dom->solid[n] ? 0.0 : feq[i];
        dom->tau[n] = 0.5 + nu0 / CS2;
    }
    dom->t = 0;
}

void orc_set_state(orc_domain* dom, const double* P, const double* tau)
{
    memcpy(dom->P, P, sizeof(double) * (size_t)(dom->L.q * dom->N));
    if (tau) memcpy(dom->tau, tau, sizeof(double) * (size_t)dom->N);
}

void orc_get_state(const orc_domain* dom, double* P, double* tau)
{
    memcpy(P, dom->P, sizeof(double) * (size_t)(dom->L.q * dom->N));
    if (tau) memcpy(tau, dom->tau, sizeof(double) * (size_t)dom->N);
}

/* Neighbour of (x,y,z) at offset -c (where the population travelling along c
 * comes from).  Returns the node index, or -1 if that place is solid or lies
 * beyond a wall face. */
static int64_t upstream_fluid(const orc_domain* dom, int x, int y, int z, const int* c)
{
    int p[3] = {x - c[0], y - c[1], z - c[2]};
    for (int a = 0; a < 3; ++a) {
        if (p[a] < 0 || p[a] >= dom->n[a]) {
            if (!dom->periodic[a]) return -1;
            p[a] = (p[a] + dom->n[a]) % dom->n[a];
        }
    }
    int64_t m = p[0] + (int64_t)dom->n[0] * (p[1] + (int64_t)dom->n[1] * p[2]);
    return dom->solid[m] ? -1 : m;
}

/* Streaming step of Eq. 10: fbar_i(x) = fpost_i(x - c_i); where x - c_i is a
 * solid node or beyond a wall, halfway bounce-back returns the node's own
 * post-collision population of the opposite direction (Sec. 4.3). */
static void pull(const orc_domain* dom, int x, int y, int z, double* fbar)
{
    int64_t n = x + (int64_t)dom->n[0] * (y + (int64_t)dom->n[1] * z);
    for (int i = 0; i < dom->L.q; ++i) {
        int64_t src = upstream_fluid(dom, x, y, z, dom->L.c[i]);
        if (src >= 0)
            fbar[i] = dom->P[i * dom->N + src];
        else
            fbar[i] = dom->P[dom->L.opp[i] * dom->N + n];
    }
}

static void collide_node(const orc_domain* dom, const double* fbar, double tau_prev,
                         double* fpost, double* tau_new, double* u_out,
                         double* nu_app, int* unyielded)
{
    double out[23];
    if (dom->rh.op == ORC_PR || dom->rh.op == ORC_PRI) {
        if (dom->rh.op == ORC_PR) collide_pr(&dom->L, &dom->rh, fbar, tau_prev, fpost, out);
        else collide_pri(&dom->L, &dom->rh, fbar, fpost, out);
        *tau_new = out[0];
        *nu_app = out[1];
        for (int a = 0; a < 3; ++a) u_out[a] = out[3 + a];
        *unyielded = (int)out[6];
    } else if (dom->rh.op == ORC_IR || dom->rh.op == ORC_IRHB) {
        collide_ir(&dom->L, &dom->rh, fbar, fpost, out);
        *tau_new = tau_prev;
        *nu_app = 0.0;
        for (int a = 0; a < 3; ++a) u_out[a] = out[a];
        *unyielded = (int)out[4];
    } else {
        collide_bgk(&dom->L, &dom->rh, fbar, fpost, out);
        *tau_new = tau_prev;
        *nu_app = dom->rh.nu_p;
        for (int a = 0; a < 3; ++a) u_out[a] = out[a];
        *unyielded = 0;
    }
}

/* Nodes are updated independently (each reads the previous state and writes
 * only its own entries), so the rows (y, z) may be shared among threads: the
 * arithmetic of every node, and hence the result, is the same for any thread
 * count. */
void orc_step(orc_domain* dom, int64_t nsteps)
{
    const int64_t rows = (int64_t)dom->n[1] * dom->n[2];
    for (int64_t s = 0; s < nsteps; ++s) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int64_t r = 0; r < rows; ++r) {
            const int y = (int)(r % dom->n[1]), z = (int)(r / dom->n[1]);
            double fbar[QMAX], fpost[QMAX], u[3], nu;
            int uy;
            for (int x = 0; x < dom->n[0]; ++x) {
                int64_t n = x + (int64_t)dom->n[0] * (y + (int64_t)dom->n[1] * z);
                if (dom->solid[n]) {
                    for (int i = 0; i < dom->L.q; ++i) dom->Pnew[i * dom->N + n] = 0.0;
                    dom->taunew[n] = dom->tau[n];
                    continue;
                }
                pull(dom, x, y, z, fbar);
                collide_node(dom, fbar, dom->tau[n], fpost, &dom->taunew[n], u, &nu, &uy);
                for (int i = 0; i < dom->L.q; ++i) dom->Pnew[i * dom->N + n] = fpost[i];
            }
        }
        double* tp = dom->P; dom->P = dom->Pnew; dom->Pnew = tp;
        double* tt = dom->tau; dom->tau = dom->taunew; dom->taunew = tt;
        dom->t++;
    }
}

int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

void orc_moments(const orc_domain* dom, double* rho, double* u, double* nu_app,
                 uint8_t* unyielded)
{
    const int64_t rows = (int64_t)dom->n[1] * dom->n[2];
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t row = 0; row < rows; ++row) {
        const int y = (int)(row % dom->n[1]), z = (int)(row / dom->n[1]);
        double fbar[QMAX], fpost[QMAX], uo[3], nu, tau_new, r, j[3];
        int uy;
        for (int x = 0; x < dom->n[0]; ++x) {
            int64_t n = x + (int64_t)dom->n[0] * (y + (int64_t)dom->n[1] * z);
            if (dom->solid[n]) {
                if (rho) rho[n] = 0.0;
                if (u) for (int a = 0; a < 3; ++a) u[a * dom->N + n] = 0.0;
                if (nu_app) nu_app[n] = 0.0;
                if (unyielded) unyielded[n] = 0;
                continue;
            }
            pull(dom, x, y, z, fbar);
            density_momentum(&dom->L, fbar, &r, j);
            collide_node(dom, fbar, dom->tau[n], fpost, &tau_new, uo, &nu, &uy);
            if (rho) rho[n] = r;
            if (u) for (int a = 0; a < 3; ++a) u[a * dom->N + n] = uo[a];
            if (nu_app) nu_app[n] = nu;
            if (unyielded) unyielded[n] = (uint8_t)uy;
        }
    }
}

void orc_monitors(const orc_domain* dom, double* out, int64_t* counts)
{
    double* rho = (double*)malloc(sizeof(double) * (size_t)dom->N);
    double* u = (double*)malloc(sizeof(double) * 3 * (size_t)dom->N);
    uint8_t* uy = (uint8_t*)malloc((size_t)dom->N);
    orc_moments(dom, rho, u, NULL, uy);
    double flux[3] = {0, 0, 0}, mass = 0.0, umax = 0.0;
    int64_t nuy = 0, nbad = 0, nfl = 0;
    for (int64_t n = 0; n < dom->N; ++n) {
        if (dom->solid[n]) continue;
        nfl++;
        double m2 = 0.0;
        int bad = !isfinite(rho[n]);
        for (int a = 0; a < 3; ++a) {
            flux[a] += u[a * dom->N + n];
            m2 += u[a * dom->N + n] * u[a * dom->N + n];
            bad |= !isfinite(u[a * dom->N + n]);
        }
        mass += rho[n];
        if (sqrt(m2) > umax) umax = sqrt(m2);
        nuy += uy[n];
        nbad += bad;
    }
    for (int a = 0; a < 3; ++a) out[a] = flux[a] / (double)dom->N;
    out[3] = mass;
    out[4] = umax;
    counts[0] = nuy;
    counts[1] = nbad;
    counts[2] = nfl;
    free(rho); free(u); free(uy);
}

/* Convergence of the velocity field between two records, the quantity the
 * steady-state criteria of Sec. 4.3 and 4.5 watch. */
void orc_residual(const orc_domain* dom, double* uprev, int record, double* out)
{
    double* u = (double*)malloc(sizeof(double) * 3 * (size_t)dom->N);
    orc_moments(dom, NULL, u, NULL, NULL);
    double num = 0.0, den = 0.0, dmax = 0.0;
    for (int64_t n = 0; n < dom->N; ++n) {
        if (dom->solid[n]) continue;
        double d2 = 0.0, u2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double ua = u[a * dom->N + n];
            const double da = ua - uprev[a * dom->N + n];
            d2 += da * da;
            u2 += ua * ua;
        }
        num += d2;
        den += u2;
        if (sqrt(d2) > dmax) dmax = sqrt(d2);
    }
    out[0] = den > 0.0 ? num / den : 0.0;
    out[1] = dmax;
    if (record)
        for (int64_t j = 0; j < 3 * dom->N; ++j) uprev[j] = dom->solid[j % dom->N] ? 0.0 : u[j];
    free(u);
}
