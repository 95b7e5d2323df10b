/*
 * lbm_oracle.h -- plain, slow FP64 CPU reference of the Bingham-fluid lattice
 * Boltzmann update of Regulski, Leonardi & Szumbarski (arXiv:1610.01388).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library; it is
 * loaded by the test-suite, by the smoke check and by the CPU-baseline leg of
 * the benchmark, never by the product path.  It shares no source, header,
 * table or helper with the HIP library.
 *
 * Conventions (all chosen here, stated so that a caller can build inputs):
 *   - node index n = x + nx*(y + ny*z), x fastest;
 *   - populations are stored as P[i*N + n] (direction-major), i in the oracle's
 *     own velocity order, returned by orc_lattice_info();
 *   - the stored state is the set of post-collision populations of the last
 *     step (time t means t collisions done); moments at time t are those of
 *     the pulled (streamed) populations that the next collision would see;
 *   - mask byte 1 = solid, 0 = fluid; non-periodic axes have a bounce-back
 *     wall half a node outside the first and last node.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_D2Q9 = 0, ORC_D3Q19 = 1, ORC_D3Q27 = 2 };
enum { ORC_PR = 0, ORC_IR = 1, ORC_BGK = 2, ORC_PRI = 3, ORC_IRHB = 4 };

/* Rheology and forcing.  op: ORC_PR (Papanastasiou-regularised, TRT + EDM,
 * explicit relaxation-time update), ORC_IR (implicitly-regularised),
 * ORC_BGK (Newtonian BGK + EDM reference, tau = 1/2 + 3 nu_p), ORC_PRI (PR
 * with the implicit relaxation-time update of Sec. 3: no state carried
 * between steps), ORC_IRHB (the implicit construction of Sec. 2.3 solved
 * for a Herschel-Bulkley fluid, as Sec. 3.2 notes it can be: nu_p is the
 * consistency K, hb_n the flow index; hb_n = 1 is the Bingham IR). */
typedef struct {
    int32_t op;
    int32_t flow_axis; /* 0: off; 1, 2, 3: the flow is known to be along x, y,
                          z and the axis-normal component is dropped from the
                          collision (Sec. 4.2.2): PR's strain rate loses d_aa,
                          IR's T loses T_aa before the deviator */
    double nu_p;      /* plastic (kinematic) viscosity, lattice units      */
    double sigma_y;   /* yield stress (per unit density), lattice units    */
    double m;         /* Papanastasiou regularisation parameter  (PR)      */
    double gamma_c;   /* strain-rate cut-off of the interpolation (PR)     */
    double lambda;    /* TRT magic number (PR)                             */
    double g[3];      /* body force per unit mass                          */
    double mrt_bulk;  /* PR / PRI: MRT relaxation rates (Sec. 2.1, Eq. 20) of */
    double mrt_even;  /* the bulk (trace) moment and of the even moments of  */
                      /* order >= 4; 0 = the shear rate (TRT).  Odd moments   */
                      /* keep the magic-number rate.  Both 0: plain TRT.      */
    double hb_n;      /* IRHB: flow index n > 0 of sigma = sigma_y + K g^n   */
} orc_rheology;

typedef struct orc_domain orc_domain;

/* Lattice tables in the oracle's order.  c is q*3 ints, w q doubles, opp q
 * ints.  Returns q, or -1 for an unknown lattice. */
int orc_lattice_info(int lattice, int* d, int* c, double* w, int* opp);

/* Second-order equilibrium of the paper (Sec. 2.1, Eq. 12). */
int orc_equilibrium(int lattice, double rho, const double* u, double* feq);

/* One collision at one node.  fbar: the q pre-collision (transformed)
 * populations.  fpost: the q post-collision populations.
 * PR: tau_prev in, out[0]=tau_new, out[1]=nu_app, out[2]=gamma_dot,
 *     out[3..5]=output velocity, out[6]=unyielded flag (stress below yield).
 * IR: out[0..2]=output velocity, out[3]=T, out[4]=unyielded flag,
 *     out[5..13]=s (3x3, row-major), out[14..22]=sigma (3x3).
 * BGK: out[0..2]=output velocity. */
int orc_collide_pr(int lattice, const orc_rheology* rh, const double* fbar,
                   double tau_prev, double* fpost, double* out);
int orc_collide_ir(int lattice, const orc_rheology* rh, const double* fbar,
                   double* fpost, double* out);
int orc_collide_bgk(int lattice, const orc_rheology* rh, const double* fbar,
                    double* fpost, double* out);
/* PRI: out as PR (out[0] = the self-consistent relaxation time).
 * IRHB: use orc_collide_ir with rh->op == ORC_IRHB (out as IR). */
int orc_collide_pri(int lattice, const orc_rheology* rh, const double* fbar,
                    double* fpost, double* out);

/* The PR apparent viscosity (Sec. 3.1, Eqs. 36-37). */
double orc_nu_app(const orc_rheology* rh, double gamma_dot, double rho);

/* Domains.  mask may be NULL (all fluid). periodic: 3 ints. */
orc_domain* orc_create(int lattice, int nx, int ny, int nz, const int* periodic,
                       const uint8_t* mask, const orc_rheology* rh);
void orc_destroy(orc_domain* dom);
/* P = f_eq(rho0, u0) at every fluid node; PR relaxation time set to the
 * zero-strain value 1/2 + 3 nu_0. */
void orc_init_equilibrium(orc_domain* dom, double rho0, const double* u0);
/* Copy in / out the stored post-collision populations (q*N, oracle order)
 * and the PR relaxation-time field (N, may be NULL). */
void orc_set_state(orc_domain* dom, const double* P, const double* tau);
void orc_get_state(const orc_domain* dom, double* P, double* tau);
/* nsteps full updates: pull-stream with bounce-back, then collide. */
void orc_step(orc_domain* dom, int64_t nsteps);
/* Threads that orc_step and orc_moments share the rows among (n > 0 sets
 * it; built without OpenMP: always 1).  Returns the count in effect.  The
 * results do not depend on it. */
int orc_set_threads(int n);
int64_t orc_time(const orc_domain* dom);
/* Moments at the current time.  rho[N], u[3*N] (component-major u[a*N+n]),
 * nu_app[N] (PR only; may be NULL), unyielded[N] (may be NULL).  Solid nodes
 * report 0. */
void orc_moments(const orc_domain* dom, double* rho, double* u, double* nu_app,
                 uint8_t* unyielded);
/* Integral monitors at the current time: out[0..2] = sum of the output
 * velocity over fluid nodes divided by all nodes (superficial velocity),
 * out[3] = total mass, out[4] = max |u|.  counts[0] = unyielded fluid nodes,
 * counts[1] = non-finite fluid nodes, counts[2] = fluid nodes. */
void orc_monitors(const orc_domain* dom, double* out, int64_t* counts);
/* Steady-state residual of the current output velocity u against a kept
 * earlier one, uprev[3*N] (component-major), over fluid nodes:
 * out[0] = sum |u - uprev|^2 / sum |u|^2 (0 when sum |u|^2 = 0),
 * out[1] = max |u - uprev|.  With record != 0, uprev is then set to u. */
void orc_residual(const orc_domain* dom, double* uprev, int record, double* out);

#ifdef __cplusplus
}
#endif
#endif
