/*
 * lbm_oracle.h -- plain FP64 CPU oracle of the phase-field lattice Boltzmann
 * method for a freezing droplet in a uniform electric field
 * (Huang, Li, Che, Chai, Wang, Shi, "Freezing dynamics of wetting droplet
 * under a uniform electric field", arXiv:2410.06657).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no source with the GPU path: its own parameter
 * struct, its own lattice tables, its own boundary rules, written straight
 * from Secs. 2-3 and Algorithm 1 of the paper.  Single threaded unless
 * orc_set_threads() is given a larger count (the threaded loops are per
 * node and independent; every reduction runs serially in row-major order,
 * so the result does not depend on the thread count).
 *
 * Grid: nodes (i, j), 0 <= i < nx, 0 <= j < ny, at x = i, y = j.  Periodic
 * in x.  Walls at y = -1/2 (cooled substrate, lower electrode) and
 * y = ny - 1/2 (upper electrode) as half-way links.  Temperatures are
 * measured from the melting point (T_m = 0).
 *
 * Every function returns 0 on success or a negative ORC_E* code.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOCONV (-2)
#define ORC_ENOMEM (-3)

/* Reading switches (bits of orc_params.readings). */
#define ORC_R_GRAD_S 1u /* include c_s^2 grad(S) in F~ of Eq. (24); off => 0 */

typedef struct orc_params {
    int nx, ny;
    /* phase field, Eqs. (2a), (3)-(5), (15)-(20) */
    double W, M, gamma;
    /* per-phase properties mixed by Eq. (1) */
    double rho_l, rho_g, rho_s;
    double mu_l, mu_g, mu_s;
    double cp_l, cp_g, cp_s;    /* specific heat per unit mass */
    double k_l, k_g, k_s;       /* thermal conductivity */
    double latent;              /* latent heat per unit mass */
    double T_w, T_g;            /* substrate and initial temperature */
    double eps_l, eps_g, eps_s; /* permittivity */
    double sig_l, sig_g, sig_s; /* conductivity */
    double phi_top, phi_bot;    /* electrode potentials */
    double theta_deg;           /* contact angle at the substrate */
    /* initial interface: shape 0 = disc (centre xc, yc, radius R0),
       shape 1 = liquid layer y < h0 */
    int shape;
    double R0, xc, yc, h0;
    /* inner potential loop: stop when the relative sweep-to-sweep change
       <= tol (tol < 0: run exactly max_sweeps sweeps) */
    double poisson_tol;
    int poisson_max_sweeps;
    unsigned readings;
} orc_params;

/* Scalar fields, one double per node, row-major [j][i]. */
enum {
    ORC_PSI = 0, ORC_UX, ORC_UY, ORC_USX, ORC_USY, ORC_P, ORC_T, ORC_H,
    ORC_FS, ORC_MDOT, ORC_PSIU_X, ORC_PSIU_Y, ORC_PHI, ORC_FL,
    ORC_NFIELDS
};
/* Population sets: [q][j][i].  ORC_POP_G_POST (read only) is the post-collision g of the
   last step, before streaming: what the enthalpy budget of the walls is written in. */
enum { ORC_POP_F = 0, ORC_POP_H = 1, ORC_POP_G = 2, ORC_POP_L = 3, ORC_POP_G_POST = 4 };

typedef struct orc_diag {
    long long step;
    double sum_psi, sum_f, sum_g;
    double V_l, V_s;          /* sum of psi*f_l and of f_s */
    double front_y;           /* f_l = 1/2 crossing on the centre column */
    double height;            /* psi = 1/2 crossing on the centre column, from the wall */
    double max_u;
    double resid;             /* last potential relative change */
    int sweeps;               /* sweeps of the last potential solve */
    int noconv;               /* potential solves that hit the sweep cap */
    double t_fre;             /* interpolated freezing step, -1 if not yet */
    double V_l0;              /* V_l at initialisation */
    int nonfinite;
    /* operator residual of the potential equation div(sigma grad phi) = 0 (Sec. 2), written
       with the isotropic stencils of Eq. (36) as grad(sigma).grad(phi) + sigma lap(phi), sigma
       mixed by Eq. (1) from the current psi and f_s: its L2 norm over the grid for the current
       phi, and for the linear electrode ramp with the same sigma (the residual the solve
       starts from; 0 when sigma is uniform) */
    double op_resid, op_resid_ramp;
} orc_diag;

typedef struct orc_state orc_state;

int  orc_set_threads(int n);
int  orc_create(const orc_params* p, orc_state** out);
void orc_destroy(orc_state* s);
int  orc_init(orc_state* s);                 /* fields, equilibria, first solve */
int  orc_step(orc_state* s, int n);          /* n full time steps */
int  orc_solve_potential(orc_state* s, double tol, int max_sweeps,
                         int* sweeps, double* resid);
int  orc_get_field(const orc_state* s, int field, double* dst);
int  orc_set_field(orc_state* s, int field, const double* src);
int  orc_get_pop(const orc_state* s, int set, double* dst);
int  orc_set_pop(orc_state* s, int set, const double* src);
int  orc_diagnostics(const orc_state* s, orc_diag* d);
/* per-step potential sweep counts recorded since init (up to cap entries) */
int  orc_sweep_log(const orc_state* s, int* dst, int cap, int* count);

/* ---- node-level pieces, exported so their moments can be pinned ---- */
void orc_node_f(double psi, double ux, double uy, double Ax, double Ay,
                double mdot, double feq[9], double F[9]);
void orc_node_h(double p, double rho, double ux, double uy, double S,
                double Ftx, double Fty, double Gx, double Gy,
                double heq[9], double R[9]);
void orc_node_g(double H, double T, double C, double Cref, double ux,
                double uy, double geq[9]);
void orc_node_l(double phi, double leq[5]);
int  orc_invert_enthalpy(const orc_params* p, double H, double psi,
                         double* T, double* fl);
/* isotropic gradient and Laplacian of a field on the grid with one of the
   oracle's ghost rules: 0 mirror, 1 wetting (psi), 2 Dirichlet (phi) */
int  orc_stencil(const orc_params* p, const double* field, int ghost,
                 double* gx, double* gy, double* lap);

#ifdef __cplusplus
}
#endif
#endif
