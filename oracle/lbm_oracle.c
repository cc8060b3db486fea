/*
 * lbm_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Follows the paper (arXiv:2410.06657) in the order of its Algorithm 1:
 *   f (phase field, Sec. 3.1, Eqs. (15)-(20)) -> bounce-back -> wetting
 *   -> psi, rho, F_s (Eqs. (20), (1), (3)-(5))
 *   -> l (electric potential, Sec. 3.4, Eqs. (31)-(34)) swept to convergence
 *   -> phi, F_e (Eqs. (34), (14))
 *   -> h (flow, Sec. 3.2, Eqs. (21)-(27)) -> bounce-back -> u, p
 *   -> g (enthalpy, Sec. 3.3, Eqs. (28)-(30)) -> Dirichlet/adiabatic walls
 *   -> T, f_l, f_s (Eq. (7)).
 * Gradients and Laplacians are the isotropic schemes of Eq. (36);
 * the time derivative of psi*u is the Euler difference of Eq. (35).
 *
 * Readings where the paper is silent or garbled (each is listed in the
 * design notes of the repository):
 *  - the interface normal is grad(psi)/|grad(psi)| and is taken as zero
 *    where |grad(psi)| <= 1e-12; the Laplacian in the chemical potential
 *    acts on psi; psi_l = 1, psi_g = 0;
 *  - div(u) in Eqs. (19)-(20) is the local volume source mdot of Eq. (2b);
 *    Eq. (20) is solved for psi: psi = sum f / (1 - mdot/2);
 *  - d/dt(psi u) = psi^n u^n - (psi u)^{n-1}, zero at the first step;
 *  - the solid force of Eq. (26) uses u_s = 0 and f_s of the previous step;
 *    the collision uses the stored u*^n, the moments use the new u*;
 *  - the c_s^2 "div S" term of F~ is c_s^2 grad(S) (switchable);
 *  - tau in Eq. (27) is the node's tau_h and R_0 its collision value;
 *  - tau_h = mu/(rho c_s^2) + 1/2 with mu and rho mixed by Eq. (1);
 *  - g carries the volumetric enthalpy rho*H; C = rho*c_p is mixed by
 *    Eq. (1) per phase; C_ref = 2 C_s C_l/(C_s + C_l) is constant;
 *    tau_g = k/(C_ref c_s^2) + 1/2; the source of Eq. (28) is weighted by
 *    omega_i and relaxed by (1 - 1/(2 tau_g));
 *  - Eq. (7) with T_s = T_l = T_m = 0; latent heat per volume
 *    rho_s*L*psi (none in the gas); f_s = psi (1 - f_l);
 *  - mdot^{n+1} = (1 - rho_s/rho_l)(f_s^{n+1} - f_s^n);
 *  - H = sum g + Q/2 with Q = C T^n mdot^n from the collision;
 *  - the loop of Algorithm 1 that runs "while the field converges" is
 *    the potential sweeps alone; h and g are updated once per step;
 *  - sweep k stops when ||phi^k - phi^{k-1}||_2 / ||phi^k||_2 <= tol;
 *  - walls: half-way bounce-back for f and h; half-way anti-bounce-back
 *    at the electrodes for l; anti-bounce-back at T_w on the substrate and
 *    bounce-back (adiabatic) at the top for g; periodic in x;
 *  - wetting: cubic wall energy, ghost psi(i,-1) = psi(i,0) +
 *    (4/W) cos(theta) psi(i,0)(1 - psi(i,0)); mirror at the top;
 *  - ghost rows of p and S mirror; of rho, eps, sigma are mixed from the
 *    ghost psi and mirrored f_s; of phi are 2 phi_wall - phi(edge);
 *  - psi is clamped to [0, 1] inside Eq. (1) and in lambda = 4 psi (1 - psi) / W of the
 *    Allen-Cahn counter term (beyond [0, 1] the printed factor changes sign, and the term
 *    would sharpen an overshoot instead of relaxing it); F_b = 0.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D2Q9, Eqs. (16)-(17): rest, four axis links (E, N, W, S), four diagonals
   (NE, NW, SW, SE). */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WQ[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
/* D2Q5, Eq. (33): rest, E, N, W, S. */
static const int LX[5] = {0, 1, 0, -1, 0};
static const int LY[5] = {0, 0, 1, 0, -1};
static const double LW[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
static const int LOPP[5] = {0, 3, 4, 1, 2};
static const double CS2 = 1.0 / 3.0;

enum { GH_MIRROR = 0, GH_WET = 1, GH_PHI = 2 };

struct orc_state {
    orc_params p;
    int nx, ny, N;
    double *f, *h, *g, *l;       /* pre-collision populations [q][N] */
    double *ft, *ht, *gt, *lt;   /* post-collision */
    double *fld[ORC_NFIELDS];
    /* per-step work arrays */
    double *pad_a, *pad_b, *pad_c, *pad_d, *pad_e; /* (ny+2)*nx padded */
    double *Fx, *Fy, *S, *tauh, *R0, *Q, *taul;
    double wet;                  /* (4/W) cos(theta) */
    double Cref, Lvol;
    long long step;
    int last_sweeps, noconv;
    double last_resid;
    double V_l0, V_prev, t_fre;
    int *log;
    int log_n, log_cap;
};

static int g_threads = 1;

int orc_set_threads(int n) {
    if (n < 1) return ORC_EINVAL;
    g_threads = n;
#ifdef _OPENMP
    omp_set_num_threads(n);
#endif
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Eq. (1): three-phase mixture with psi clamped to [0, 1].            */
static double mix(double chs, double chl, double chg, double psi, double fs) {
    double pc = psi < 0 ? 0 : (psi > 1 ? 1 : psi);
    return fs * chs + (1 - fs) * pc * chl + (1 - fs) * (1 - pc) * chg;
}
static double clamp01(double x) { return x < 0 ? 0 : (x > 1 ? 1 : x); }

/* ------------------------------------------------------------------ */
/* Node-level equilibria and forcing terms.                            */

/* Eqs. (18)-(19). A = d/dt(psi u) + c_s^2 lambda n. */
void orc_node_f(double psi, double ux, double uy, double Ax, double Ay,
                double mdot, double feq[9], double F[9]) {
    for (int q = 0; q < 9; q++) {
        double cu = CX[q] * ux + CY[q] * uy;
        feq[q] = WQ[q] * psi * (1 + cu / CS2);
        F[q] = WQ[q] * (CX[q] * Ax + CY[q] * Ay) / CS2 + WQ[q] * psi * mdot;
    }
}

/* Eqs. (22)-(24). (Ftx, Fty) = F~, (Gx, Gy) = F + rho*f_solid. */
void orc_node_h(double p, double rho, double ux, double uy, double S,
                double Ftx, double Fty, double Gx, double Gy,
                double heq[9], double R[9]) {
    double uu = ux * ux + uy * uy;
    double uF = ux * Ftx + uy * Fty;
    for (int q = 0; q < 9; q++) {
        double cu = CX[q] * ux + CY[q] * uy;
        double s = WQ[q] * (cu / CS2 + cu * cu / (2 * CS2 * CS2) - uu / (2 * CS2));
        if (q == 0)
            heq[q] = p / CS2 * (WQ[q] - 1) + rho * s;
        else
            heq[q] = p / CS2 * WQ[q] + rho * s;
        double cF = CX[q] * Ftx + CY[q] * Fty;
        double cG = CX[q] * Gx + CY[q] * Gy;
        /* (u F~ + F~ u) : (c c - c_s^2 I) / (2 c_s^4) */
        double sec = (2 * cu * cF - 2 * CS2 * uF) / (2 * CS2 * CS2);
        R[q] = WQ[q] * (S + cG / CS2 + sec);
    }
}

/* Eq. (29); C_p (C_ref/C_p) is written as C_ref. */
void orc_node_g(double H, double T, double C, double Cref, double ux,
                double uy, double geq[9]) {
    double uu = ux * ux + uy * uy;
    geq[0] = H - Cref * T + WQ[0] * (Cref * T - C * T * uu / (2 * CS2));
    for (int q = 1; q < 9; q++) {
        double cu = CX[q] * ux + CY[q] * uy;
        geq[q] = WQ[q] * (Cref * T + C * T * (cu / CS2 + (cu * cu - CS2 * uu) / (2 * CS2 * CS2)));
    }
}

/* Eq. (32). */
void orc_node_l(double phi, double leq[5]) {
    leq[0] = (LW[0] - 1) * phi;
    for (int q = 1; q < 5; q++) leq[q] = LW[q] * phi;
}

static void phase_caps(const orc_params* p, double* Cs, double* Cl, double* Cg) {
    *Cs = p->rho_s * p->cp_s;
    *Cl = p->rho_l * p->cp_l;
    *Cg = p->rho_g * p->cp_g;
}

/* Eq. (7) on the volumetric enthalpy with T_s = T_l = 0. */
int orc_invert_enthalpy(const orc_params* p, double H, double psi, double* T,
                        double* fl) {
    double Cs, Cl, Cg;
    phase_caps(p, &Cs, &Cl, &Cg);
    double pc = clamp01(psi);
    double Leff = pc * p->rho_s * p->latent;
    double Csol = mix(Cs, Cl, Cg, pc, pc); /* the node with all its liquid frozen */
    double Cliq = mix(Cs, Cl, Cg, pc, 0);
    if (H < 0) {
        *fl = 0;
        *T = H / Csol;
    } else if (H <= Leff) {
        *fl = Leff > 0 ? H / Leff : 1;
        *T = 0;
    } else {
        *fl = 1;
        *T = (H - Leff) / Cliq;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Ghost rows and stencils.                                            */

static inline int wrapx(int i, int nx) {
    i %= nx;
    return i < 0 ? i + nx : i;
}

/* Copy field into a padded array of rows -1..ny (row r = j + 1) with the
   given ghost rule. */
static void pad_field(const orc_state* s, const double* src, int rule, double* dst) {
    int nx = s->nx, ny = s->ny;
    memcpy(dst + nx, src, sizeof(double) * (size_t)s->N);
    for (int i = 0; i < nx; i++) {
        double b = src[i], t = src[(size_t)(ny - 1) * nx + i];
        double gb, gt;
        if (rule == GH_WET) {
            gb = b + s->wet * b * (1 - b);
            gt = t; /* 90 degrees at the top */
        } else if (rule == GH_PHI) {
            gb = 2 * s->p.phi_bot - b;
            gt = 2 * s->p.phi_top - t;
        } else {
            gb = b;
            gt = t;
        }
        dst[i] = gb;
        dst[(size_t)(ny + 1) * nx + i] = gt;
    }
}

/* Eq. (36a) and (36b) at interior node (i, j) of a padded array. */
static void stencil_at(const orc_state* s, const double* P, int i, int j,
                       double* gx, double* gy, double* lap) {
    int nx = s->nx;
    double c = P[(size_t)(j + 1) * nx + i];
    double sx = 0, sy = 0, sl = 0;
    for (int q = 1; q < 9; q++) {
        double v = P[(size_t)(j + 1 + CY[q]) * nx + wrapx(i + CX[q], nx)];
        sx += WQ[q] * CX[q] * v;
        sy += WQ[q] * CY[q] * v;
        sl += 2 * WQ[q] * (v - c);
    }
    if (gx) *gx = sx / CS2;
    if (gy) *gy = sy / CS2;
    if (lap) *lap = sl / CS2;
}

int orc_stencil(const orc_params* p, const double* field, int ghost,
                double* gx, double* gy, double* lap) {
    if (!p || p->nx < 1 || p->ny < 1) return ORC_EINVAL;
    orc_state tmp;
    memset(&tmp, 0, sizeof tmp);
    tmp.p = *p;
    tmp.nx = p->nx;
    tmp.ny = p->ny;
    tmp.N = p->nx * p->ny;
    tmp.wet = 4.0 / p->W * cos(p->theta_deg * M_PI / 180.0);
    double* P = malloc(sizeof(double) * (size_t)(p->ny + 2) * p->nx);
    if (!P) return ORC_ENOMEM;
    pad_field(&tmp, field, ghost, P);
    for (int j = 0; j < p->ny; j++)
        for (int i = 0; i < p->nx; i++) {
            size_t n = (size_t)j * p->nx + i;
            stencil_at(&tmp, P, i, j, gx ? gx + n : 0, gy ? gy + n : 0, lap ? lap + n : 0);
        }
    free(P);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* State management.                                                   */

static int validate(const orc_params* p) {
    if (p->nx < 2 || p->ny < 3) return ORC_EINVAL;
    if (!(p->W > 0) || !(p->M > 0) || !(p->gamma >= 0)) return ORC_EINVAL;
    if (!(p->rho_l > 0) || !(p->rho_g > 0) || !(p->rho_s > 0)) return ORC_EINVAL;
    if (!(p->mu_l > 0) || !(p->mu_g > 0) || !(p->mu_s > 0)) return ORC_EINVAL;
    if (!(p->cp_l > 0) || !(p->cp_g > 0) || !(p->cp_s > 0)) return ORC_EINVAL;
    if (!(p->k_l > 0) || !(p->k_g > 0) || !(p->k_s > 0)) return ORC_EINVAL;
    if (!(p->sig_l > 0) || !(p->sig_g > 0) || !(p->sig_s > 0)) return ORC_EINVAL;
    if (!(p->latent >= 0)) return ORC_EINVAL;
    if (p->poisson_max_sweeps < 1) return ORC_EINVAL;
    return ORC_OK;
}

void orc_destroy(orc_state* s) {
    if (!s) return;
    double* arrs[] = {s->f, s->h, s->g, s->l, s->ft, s->ht, s->gt, s->lt,
                      s->pad_a, s->pad_b, s->pad_c, s->pad_d, s->pad_e,
                      s->Fx, s->Fy, s->S, s->tauh, s->R0, s->Q, s->taul};
    for (size_t k = 0; k < sizeof arrs / sizeof arrs[0]; k++) free(arrs[k]);
    for (int k = 0; k < ORC_NFIELDS; k++) free(s->fld[k]);
    free(s->log);
    free(s);
}

int orc_create(const orc_params* p, orc_state** out) {
    if (!p || !out) return ORC_EINVAL;
    int rc = validate(p);
    if (rc) return rc;
    orc_state* s = calloc(1, sizeof *s);
    if (!s) return ORC_ENOMEM;
    s->p = *p;
    s->nx = p->nx;
    s->ny = p->ny;
    s->N = p->nx * p->ny;
    size_t N = (size_t)s->N, NP = (size_t)(p->ny + 2) * p->nx;
    int bad = 0;
#define ALLOC(ptr, cnt) do { ptr = calloc((cnt), sizeof(double)); if (!ptr) bad = 1; } while (0)
    ALLOC(s->f, 9 * N); ALLOC(s->h, 9 * N); ALLOC(s->g, 9 * N); ALLOC(s->l, 5 * N);
    ALLOC(s->ft, 9 * N); ALLOC(s->ht, 9 * N); ALLOC(s->gt, 9 * N); ALLOC(s->lt, 5 * N);
    ALLOC(s->pad_a, NP); ALLOC(s->pad_b, NP); ALLOC(s->pad_c, NP); ALLOC(s->pad_d, NP); ALLOC(s->pad_e, NP);
    ALLOC(s->Fx, N); ALLOC(s->Fy, N); ALLOC(s->S, N); ALLOC(s->tauh, N); ALLOC(s->R0, N);
    ALLOC(s->Q, N); ALLOC(s->taul, N);
    for (int k = 0; k < ORC_NFIELDS; k++) ALLOC(s->fld[k], N);
#undef ALLOC
    s->log_cap = 1 << 16;
    s->log = calloc((size_t)s->log_cap, sizeof(int));
    if (bad || !s->log) {
        orc_destroy(s);
        return ORC_ENOMEM;
    }
    s->wet = 4.0 / p->W * cos(p->theta_deg * M_PI / 180.0);
    double Cs, Cl, Cg;
    phase_caps(p, &Cs, &Cl, &Cg);
    s->Cref = 2 * Cs * Cl / (Cs + Cl);
    s->Lvol = p->rho_s * p->latent;
    s->t_fre = -1;
    *out = s;
    return ORC_OK;
}

static void log_sweeps(orc_state* s, int k) {
    if (s->log_n < s->log_cap) s->log[s->log_n] = k;
    s->log_n++;
}

/* Sum of psi*f_l over the grid, row-major. */
static double liquid_volume(const orc_state* s) {
    const double* psi = s->fld[ORC_PSI];
    const double* fl = s->fld[ORC_FL];
    double v = 0;
    for (int n = 0; n < s->N; n++) v += clamp01(psi[n]) * fl[n];
    return v;
}

/* ------------------------------------------------------------------ */
/* Electric potential, Eqs. (31)-(34), swept until the relative change  */
/* of phi between sweeps is <= tol, testing from sweep min_sweeps on.  */
static int solve_potential(orc_state* s, double tol, int min_sweeps, int max_sweeps,
                           int* sweeps, double* resid) {
    if (!s || max_sweeps < 1) return ORC_EINVAL;
    const orc_params* p = &s->p;
    int nx = s->nx, ny = s->ny, N = s->N;
    double* psi = s->fld[ORC_PSI];
    double* fs = s->fld[ORC_FS];
    double* phi = s->fld[ORC_PHI];
    double* l = s->l;
    double* lt = s->lt;
    /* tau_l = sigma/c_s^2 + 1/2 with sigma from Eq. (1). */
    for (int n = 0; n < N; n++)
        s->taul[n] = mix(p->sig_s, p->sig_l, p->sig_g, psi[n], fs[n]) / CS2 + 0.5;
    int k = 0;
    double r = 0;
    int rc = ORC_OK;
    for (;;) {
        k++;
        /* collision with the node's current phi */
#pragma omp parallel for schedule(static)
        for (int n = 0; n < N; n++) {
            double ph = 0;
            for (int q = 1; q < 5; q++) ph += l[(size_t)q * N + n];
            ph /= (1 - LW[0]);
            double leq[5];
            orc_node_l(ph, leq);
            for (int q = 0; q < 5; q++) {
                double v = l[(size_t)q * N + n];
                lt[(size_t)q * N + n] = v - (v - leq[q]) / s->taul[n];
            }
        }
        /* streaming with anti-bounce-back at the electrodes */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                int n = j * nx + i;
                for (int q = 0; q < 5; q++) {
                    int jj = j - LY[q];
                    if (jj < 0)
                        l[(size_t)q * N + n] = -lt[(size_t)LOPP[q] * N + n] + 2 * LW[q] * p->phi_bot;
                    else if (jj >= ny)
                        l[(size_t)q * N + n] = -lt[(size_t)LOPP[q] * N + n] + 2 * LW[q] * p->phi_top;
                    else
                        l[(size_t)q * N + n] = lt[(size_t)q * N + (size_t)jj * nx + wrapx(i - LX[q], nx)];
                }
            }
        /* new moment and the relative change, summed row-major */
        double d2 = 0, p2 = 0;
        for (int n = 0; n < N; n++) {
            double ph = 0;
            for (int q = 1; q < 5; q++) ph += l[(size_t)q * N + n];
            ph /= (1 - LW[0]);
            double d = ph - phi[n];
            d2 += d * d;
            p2 += ph * ph;
            phi[n] = ph;
        }
        r = d2 == 0 ? 0 : (p2 > 0 ? sqrt(d2) / sqrt(p2) : INFINITY);
        if (tol >= 0 && k >= min_sweeps && r <= tol) break;
        if (k >= max_sweeps) {
            if (tol >= 0) rc = ORC_ENOCONV;
            break;
        }
    }
    s->last_sweeps = k;
    s->last_resid = r;
    if (rc == ORC_ENOCONV) s->noconv++;
    if (sweeps) *sweeps = k;
    if (resid) *resid = r;
    return rc;
}

int orc_solve_potential(orc_state* s, double tol, int max_sweeps, int* sweeps,
                        double* resid) {
    return solve_potential(s, tol, 1, max_sweeps, sweeps, resid);
}

/* ------------------------------------------------------------------ */
/* Initialisation (Algorithm 1, first block).                          */
int orc_init(orc_state* s) {
    if (!s) return ORC_EINVAL;
    const orc_params* p = &s->p;
    int nx = s->nx, ny = s->ny, N = s->N;
    double Cs, Cl, Cg;
    phase_caps(p, &Cs, &Cl, &Cg);
    for (int k = 0; k < ORC_NFIELDS; k++) memset(s->fld[k], 0, sizeof(double) * (size_t)N);
    double* psi = s->fld[ORC_PSI];
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int n = j * nx + i;
            double v;
            if (p->shape == 1) {
                /* liquid layer of thickness h0 above the wall at y = -1/2 */
                v = 0.5 * (1 + tanh(2 * (p->h0 - 0.5 - j) / p->W));
            } else {
                double dx = i - p->xc;
                dx -= nx * floor(dx / nx + 0.5); /* nearest periodic image */
                double dy = j - p->yc;
                double r = sqrt(dx * dx + dy * dy);
                v = 0.5 * (1 + tanh(2 * (p->R0 - r) / p->W));
            }
            psi[n] = v;
            double C = mix(Cs, Cl, Cg, v, 0);
            double H = C * p->T_g + clamp01(v) * s->Lvol; /* fully liquid */
            double T, fl;
            orc_invert_enthalpy(p, H, v, &T, &fl);
            s->fld[ORC_H][n] = H;
            s->fld[ORC_T][n] = T;
            s->fld[ORC_FL][n] = fl;
            s->fld[ORC_FS][n] = clamp01(v) * (1 - fl);
            s->fld[ORC_PHI][n] = p->phi_bot + (p->phi_top - p->phi_bot) * (j + 0.5) / ny;
        }
    for (int n = 0; n < N; n++) {
        double feq[9], F[9], heq[9], R[9], geq[9], leq[5];
        double v = psi[n];
        double rho = mix(p->rho_s, p->rho_l, p->rho_g, v, s->fld[ORC_FS][n]);
        double C = mix(Cs, Cl, Cg, v, s->fld[ORC_FS][n]);
        orc_node_f(v, 0, 0, 0, 0, 0, feq, F);
        orc_node_h(0, rho, 0, 0, 0, 0, 0, 0, 0, heq, R);
        orc_node_g(s->fld[ORC_H][n], s->fld[ORC_T][n], C, s->Cref, 0, 0, geq);
        orc_node_l(s->fld[ORC_PHI][n], leq);
        for (int q = 0; q < 9; q++) {
            s->f[(size_t)q * N + n] = feq[q];
            s->h[(size_t)q * N + n] = heq[q];
            s->g[(size_t)q * N + n] = geq[q];
        }
        for (int q = 0; q < 5; q++) s->l[(size_t)q * N + n] = leq[q];
    }
    s->step = 0;
    s->noconv = 0;
    s->log_n = 0;
    s->t_fre = -1;
    /* The populations start at equilibrium: a first sweep of a linear ramp
       changes nothing, so the stopping test only counts from sweep 2 here. */
    int k = 0;
    int rc = solve_potential(s, p->poisson_tol, 2, p->poisson_max_sweeps, &k, NULL);
    log_sweeps(s, k);
    s->V_l0 = liquid_volume(s);
    s->V_prev = s->V_l0;
    return rc == ORC_ENOCONV ? ORC_OK : rc;
}

/* ------------------------------------------------------------------ */
/* One time step (Algorithm 1, main loop body).                        */
static void stream9(const orc_state* s, const double* src, double* dst, int kind) {
    /* kind 0: bounce-back at both walls; kind 1: anti-bounce-back at the
       bottom wall with value 2 w C_ref T_w, bounce-back at the top */
    int nx = s->nx, ny = s->ny;
    size_t N = (size_t)s->N;
    double wallv = s->Cref * s->p.T_w;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            size_t n = (size_t)j * nx + i;
            for (int q = 0; q < 9; q++) {
                int jj = j - CY[q];
                double v;
                if (jj < 0)
                    v = kind == 1 ? -src[OPP[q] * N + n] + 2 * WQ[q] * wallv : src[OPP[q] * N + n];
                else if (jj >= ny)
                    v = src[OPP[q] * N + n];
                else
                    v = src[q * N + (size_t)jj * nx + wrapx(i - CX[q], nx)];
                dst[q * N + n] = v;
            }
        }
}

static void step_once(orc_state* s) {
    const orc_params* p = &s->p;
    int nx = s->nx, ny = s->ny, N = s->N;
    double Cs, Cl, Cg;
    phase_caps(p, &Cs, &Cl, &Cg);
    double* psi = s->fld[ORC_PSI];
    double* ux = s->fld[ORC_UX];
    double* uy = s->fld[ORC_UY];
    double* usx = s->fld[ORC_USX];
    double* usy = s->fld[ORC_USY];
    double* pr = s->fld[ORC_P];
    double* T = s->fld[ORC_T];
    double* H = s->fld[ORC_H];
    double* fs = s->fld[ORC_FS];
    double* md = s->fld[ORC_MDOT];
    double* pux = s->fld[ORC_PSIU_X];
    double* puy = s->fld[ORC_PSIU_Y];
    double* phi = s->fld[ORC_PHI];
    double* fl = s->fld[ORC_FL];
    const double tauf = p->M / CS2 + 0.5;
    const double kap = 1.5 * p->gamma * p->W;  /* Eq. (5) */
    const double beta = 12 * p->gamma / p->W;

    /* 1. f collision, Eqs. (15), (18), (19), (35), with psi^n, u^n. */
    double* Ppsi = s->pad_a;
    pad_field(s, psi, GH_WET, Ppsi);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int n = j * nx + i;
            double gx, gy;
            stencil_at(s, Ppsi, i, j, &gx, &gy, NULL);
            double mag = sqrt(gx * gx + gy * gy);
            double nxv = 0, nyv = 0;
            if (mag > 1e-12) {
                nxv = gx / mag;
                nyv = gy / mag;
            }
            double ps = psi[n];
            /* psi clamped to [0, 1] in lambda as in Eq. (1): outside it the printed factor
               changes sign and the counter term would steepen instead of relax */
            double pcl = clamp01(ps);
            double lam = 4 * pcl * (1 - pcl) / p->W;
            double Ax = (ps * ux[n] - pux[n]) + CS2 * lam * nxv;
            double Ay = (ps * uy[n] - puy[n]) + CS2 * lam * nyv;
            double feq[9], F[9];
            orc_node_f(ps, ux[n], uy[n], Ax, Ay, md[n], feq, F);
            for (int q = 0; q < 9; q++) {
                double v = s->f[(size_t)q * N + n];
                s->ft[(size_t)q * N + n] = v - (v - feq[q]) / tauf + (1 - 0.5 / tauf) * F[q];
            }
            pux[n] = ps * ux[n];
            puy[n] = ps * uy[n];
        }
    /* 2. streaming with half-way bounce-back. */
    stream9(s, s->ft, s->f, 0);
    /* 3. psi^{n+1} from Eq. (20); properties (Eq. (1)) and F_s (Eqs. (3)-(5)). */
    for (int n = 0; n < N; n++) {
        double sum = 0;
        for (int q = 0; q < 9; q++) sum += s->f[(size_t)q * N + n];
        psi[n] = sum / (1 - 0.5 * md[n]);
    }
    pad_field(s, psi, GH_WET, Ppsi);
    double* Pfs = s->pad_b;
    pad_field(s, fs, GH_MIRROR, Pfs);
    double* Prho = s->pad_c;
    double* Peps = s->pad_d;
    size_t NP = (size_t)(ny + 2) * nx;
    for (size_t r = 0; r < NP; r++) {
        Prho[r] = mix(p->rho_s, p->rho_l, p->rho_g, Ppsi[r], Pfs[r]);
        Peps[r] = mix(p->eps_s, p->eps_l, p->eps_g, Ppsi[r], Pfs[r]);
    }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int n = j * nx + i;
            double gx, gy, lap;
            stencil_at(s, Ppsi, i, j, &gx, &gy, &lap);
            double ps = psi[n];
            double mu = 4 * beta * ps * (ps - 1) * (ps - 0.5) - kap * lap;
            s->Fx[n] = mu * gx;
            s->Fy[n] = mu * gy;
        }
    /* 4. potential to convergence. */
    int k = 0;
    solve_potential(s, p->poisson_tol, 1, p->poisson_max_sweeps, &k, NULL);
    log_sweeps(s, k);
    /* 5. electric force, Eq. (14), q_v = div(eps E). */
    double* Pphi = s->pad_e;
    pad_field(s, phi, GH_PHI, Pphi);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int n = j * nx + i;
            double gpx, gpy, lphi, gex, gey;
            stencil_at(s, Pphi, i, j, &gpx, &gpy, &lphi);
            stencil_at(s, Peps, i, j, &gex, &gey, NULL);
            double eps = Peps[(size_t)(j + 1) * nx + i];
            double Ex = -gpx, Ey = -gpy;
            double qv = -(gex * gpx + gey * gpy + eps * lphi);
            double E2 = Ex * Ex + Ey * Ey;
            s->Fx[n] += qv * Ex - 0.5 * E2 * gex;
            s->Fy[n] += qv * Ey - 0.5 * E2 * gey;
        }
    /* 6. h collision, Eqs. (21)-(24). S = rho mdot + u . grad(rho). */
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int n = j * nx + i;
            double grx, gry;
            stencil_at(s, Prho, i, j, &grx, &gry, NULL);
            s->S[n] = Prho[(size_t)(j + 1) * nx + i] * md[n] + ux[n] * grx + uy[n] * gry;
        }
    double* PS = s->pad_e; /* phi padding no longer needed */
    pad_field(s, s->S, GH_MIRROR, PS);
    double* Pp = s->pad_b; /* f_s padding no longer needed */
    pad_field(s, pr, GH_MIRROR, Pp);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int n = j * nx + i;
            double rho = Prho[(size_t)(j + 1) * nx + i];
            double mu = mix(p->mu_s, p->mu_l, p->mu_g, psi[n], fs[n]);
            double tauh = mu / (rho * CS2) + 0.5;
            double grx, gry, gpx, gpy, gsx = 0, gsy = 0;
            stencil_at(s, Prho, i, j, &grx, &gry, NULL);
            stencil_at(s, Pp, i, j, &gpx, &gpy, NULL);
            if (p->readings & ORC_R_GRAD_S) stencil_at(s, PS, i, j, &gsx, &gsy, NULL);
            double Ftx = s->Fx[n] - gpx + CS2 * grx + CS2 * gsx;
            double Fty = s->Fy[n] - gpy + CS2 * gry + CS2 * gsy;
            double fsx = fs[n] * (0 - usx[n]); /* solid force, Eq. (26) text */
            double fsy = fs[n] * (0 - usy[n]);
            double Gx = s->Fx[n] + rho * fsx;
            double Gy = s->Fy[n] + rho * fsy;
            double heq[9], R[9];
            orc_node_h(pr[n], rho, ux[n], uy[n], s->S[n], Ftx, Fty, Gx, Gy, heq, R);
            for (int q = 0; q < 9; q++) {
                double v = s->h[(size_t)q * N + n];
                s->ht[(size_t)q * N + n] = v - (v - heq[q]) / tauh + (1 - 0.5 / tauh) * R[q];
            }
            s->tauh[n] = tauh;
            s->R0[n] = R[0];
        }
    /* 7. streaming with bounce-back, then u*, u, p (Eqs. (25)-(27)). */
    stream9(s, s->ht, s->h, 0);
#pragma omp parallel for schedule(static)
    for (int n = 0; n < N; n++) {
        double sx = 0, sy = 0, s0 = 0;
        for (int q = 0; q < 9; q++) {
            double v = s->h[(size_t)q * N + n];
            sx += CX[q] * v;
            sy += CY[q] * v;
            if (q) s0 += v;
        }
        int j = n / nx, i = n % nx;
        double rho = Prho[(size_t)(j + 1) * nx + i];
        double ax = (sx + 0.5 * s->Fx[n]) / rho;
        double ay = (sy + 0.5 * s->Fy[n]) / rho;
        usx[n] = ax;
        usy[n] = ay;
        ux[n] = ax + 0.5 * fs[n] * (0 - ax);
        uy[n] = ay + 0.5 * fs[n] * (0 - ay);
        double uu = ux[n] * ux[n] + uy[n] * uy[n];
        double s0u = WQ[0] * (-uu / (2 * CS2));
        pr[n] = CS2 / (1 - WQ[0]) * (s0 + 0.5 * s->S[n] + s->tauh[n] * s->R0[n] + rho * s0u);
    }
    /* 8. g collision, Eqs. (28)-(29), with u^{n+1}, H^n, T^n. */
#pragma omp parallel for schedule(static)
    for (int n = 0; n < N; n++) {
        double C = mix(Cs, Cl, Cg, psi[n], fs[n]);
        double kth = mix(p->k_s, p->k_l, p->k_g, psi[n], fs[n]);
        double taug = kth / (s->Cref * CS2) + 0.5;
        double Qn = C * T[n] * md[n];
        double geq[9];
        orc_node_g(H[n], T[n], C, s->Cref, ux[n], uy[n], geq);
        for (int q = 0; q < 9; q++) {
            double v = s->g[(size_t)q * N + n];
            s->gt[(size_t)q * N + n] = v - (v - geq[q]) / taug + (1 - 0.5 / taug) * WQ[q] * Qn;
        }
        s->Q[n] = Qn;
    }
    /* 9. streaming: substrate at T_w, adiabatic top; H^{n+1} by Eq. (30). */
    stream9(s, s->gt, s->g, 1);
    /* 10. Eq. (7): T, f_l; f_s^{n+1} and the volume source mdot^{n+1}. */
    const double shrink = 1 - p->rho_s / p->rho_l;
#pragma omp parallel for schedule(static)
    for (int n = 0; n < N; n++) {
        double sum = 0;
        for (int q = 0; q < 9; q++) sum += s->g[(size_t)q * N + n];
        H[n] = sum + 0.5 * s->Q[n];
        double Tn, fln;
        orc_invert_enthalpy(p, H[n], psi[n], &Tn, &fln);
        T[n] = Tn;
        fl[n] = fln;
        double fsn = clamp01(psi[n]) * (1 - fln);
        md[n] = shrink * (fsn - fs[n]);
        fs[n] = fsn;
    }
    s->step++;
    /* freezing time: first step with V_l <= 1% of its initial value */
    double V = liquid_volume(s);
    if (s->t_fre < 0 && s->V_l0 > 0 && V <= 0.01 * s->V_l0) {
        double thr = 0.01 * s->V_l0;
        double dv = s->V_prev - V;
        s->t_fre = (double)(s->step - 1) + (dv > 0 ? (s->V_prev - thr) / dv : 1.0);
    }
    s->V_prev = V;
}

int orc_step(orc_state* s, int n) {
    if (!s || n < 0) return ORC_EINVAL;
    for (int k = 0; k < n; k++) step_once(s);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Field access and diagnostics.                                       */
int orc_get_field(const orc_state* s, int field, double* dst) {
    if (!s || !dst || field < 0 || field >= ORC_NFIELDS) return ORC_EINVAL;
    memcpy(dst, s->fld[field], sizeof(double) * (size_t)s->N);
    return ORC_OK;
}
int orc_set_field(orc_state* s, int field, const double* src) {
    if (!s || !src || field < 0 || field >= ORC_NFIELDS) return ORC_EINVAL;
    memcpy(s->fld[field], src, sizeof(double) * (size_t)s->N);
    return ORC_OK;
}
static double* pop_ptr(const orc_state* s, int set, int* nq) {
    switch (set) {
        case ORC_POP_F: *nq = 9; return s->f;
        case ORC_POP_H: *nq = 9; return s->h;
        case ORC_POP_G: *nq = 9; return s->g;
        case ORC_POP_L: *nq = 5; return s->l;
        case ORC_POP_G_POST: *nq = 9; return s->gt;
        default: return NULL;
    }
}
int orc_get_pop(const orc_state* s, int set, double* dst) {
    int nq = 0;
    double* ptr = s ? pop_ptr(s, set, &nq) : NULL;
    if (!ptr || !dst) return ORC_EINVAL;
    memcpy(dst, ptr, sizeof(double) * (size_t)nq * s->N);
    return ORC_OK;
}
int orc_set_pop(orc_state* s, int set, const double* src) {
    if (set == ORC_POP_G_POST) return ORC_EINVAL; /* a record of the last step, not state */
    int nq = 0;
    double* ptr = s ? pop_ptr(s, set, &nq) : NULL;
    if (!ptr || !src) return ORC_EINVAL;
    memcpy(ptr, src, sizeof(double) * (size_t)nq * s->N);
    return ORC_OK;
}
int orc_sweep_log(const orc_state* s, int* dst, int cap, int* count) {
    if (!s) return ORC_EINVAL;
    int n = s->log_n < s->log_cap ? s->log_n : s->log_cap;
    if (dst)
        for (int k = 0; k < n && k < cap; k++) dst[k] = s->log[k];
    if (count) *count = s->log_n;
    return ORC_OK;
}

/* ||div(sigma grad phi)|| of the potential equation (Sec. 2) in the discrete form of Eq. (36):
   grad(sigma).grad(phi) + sigma lap(phi) at every node, with sigma mixed by Eq. (1) from the
   current psi and f_s (ghost rows: psi by the wetting rule, f_s mirrored, phi Dirichlet at the
   electrodes).  *ramp gets the same norm for the linear electrode ramp. */
static int operator_residual(const orc_state* s, double* res, double* ramp) {
    const orc_params* p = &s->p;
    int nx = s->nx, ny = s->ny;
    size_t NP = (size_t)(ny + 2) * nx;
    double* Ppsi = malloc(sizeof(double) * NP);
    double* Pfs = malloc(sizeof(double) * NP);
    double* Pphi = malloc(sizeof(double) * NP);
    double* Plin = malloc(sizeof(double) * NP);
    double* lin = malloc(sizeof(double) * (size_t)s->N);
    if (!Ppsi || !Pfs || !Pphi || !Plin || !lin) {
        free(Ppsi); free(Pfs); free(Pphi); free(Plin); free(lin);
        return ORC_ENOMEM;
    }
    pad_field(s, s->fld[ORC_PSI], GH_WET, Ppsi);
    pad_field(s, s->fld[ORC_FS], GH_MIRROR, Pfs);
    pad_field(s, s->fld[ORC_PHI], GH_PHI, Pphi);
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++)
            lin[(size_t)j * nx + i] = p->phi_bot + (p->phi_top - p->phi_bot) * (j + 0.5) / ny;
    pad_field(s, lin, GH_PHI, Plin);
    /* sigma on the padded grid (reuses the f_s array) */
    for (size_t r = 0; r < NP; r++) Pfs[r] = mix(p->sig_s, p->sig_l, p->sig_g, Ppsi[r], Pfs[r]);
    double a = 0, b = 0;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            double gsx, gsy, gpx, gpy, lap, glx, gly, llap;
            stencil_at(s, Pfs, i, j, &gsx, &gsy, NULL);
            stencil_at(s, Pphi, i, j, &gpx, &gpy, &lap);
            stencil_at(s, Plin, i, j, &glx, &gly, &llap);
            double sg = Pfs[(size_t)(j + 1) * nx + i];
            double v = gsx * gpx + gsy * gpy + sg * lap;
            double w = gsx * glx + gsy * gly + sg * llap;
            a += v * v;
            b += w * w;
        }
    *res = sqrt(a);
    *ramp = sqrt(b);
    free(Ppsi); free(Pfs); free(Pphi); free(Plin); free(lin);
    return ORC_OK;
}

int orc_diagnostics(const orc_state* s, orc_diag* d) {
    if (!s || !d) return ORC_EINVAL;
    memset(d, 0, sizeof *d);
    int nx = s->nx, ny = s->ny, N = s->N;
    const double* psi = s->fld[ORC_PSI];
    const double* fl = s->fld[ORC_FL];
    const double* fs = s->fld[ORC_FS];
    const double* ux = s->fld[ORC_UX];
    const double* uy = s->fld[ORC_UY];
    d->step = s->step;
    for (int n = 0; n < N; n++) {
        d->sum_psi += psi[n];
        d->V_l += clamp01(psi[n]) * fl[n];
        d->V_s += fs[n];
        double um = sqrt(ux[n] * ux[n] + uy[n] * uy[n]);
        if (um > d->max_u) d->max_u = um;
        double chk = psi[n] + ux[n] + uy[n] + s->fld[ORC_P][n] + s->fld[ORC_T][n] + s->fld[ORC_PHI][n];
        if (!isfinite(chk)) d->nonfinite = 1;
    }
    for (int q = 0; q < 9; q++)
        for (int n = 0; n < N; n++) d->sum_f += s->f[(size_t)q * N + n];
    for (int q = 0; q < 9; q++)
        for (int n = 0; n < N; n++) d->sum_g += s->g[(size_t)q * N + n];
    /* centre column: droplet height (psi = 1/2) and freezing front (f_l = 1/2) */
    int ic = nx / 2;
    double height = 0;
    for (int j = ny - 1; j >= 0; j--) {
        double a = psi[(size_t)j * nx + ic];
        if (a >= 0.5) {
            if (j == ny - 1) {
                height = ny;
            } else {
                double b = psi[(size_t)(j + 1) * nx + ic];
                height = j + (a - 0.5) / (a - b) + 0.5;
            }
            break;
        }
    }
    double front = 0;
    if (psi[ic] >= 0.5) {
        front = height;
        for (int j = 0; j < ny && psi[(size_t)j * nx + ic] >= 0.5; j++) {
            double a = fl[(size_t)j * nx + ic];
            if (a >= 0.5) {
                if (j == 0) {
                    front = 0;
                } else {
                    double b = fl[(size_t)(j - 1) * nx + ic];
                    front = (j - 1) + (0.5 - b) / (a - b) + 0.5;
                }
                break;
            }
        }
    }
    d->height = height;
    d->front_y = front;
    d->resid = s->last_resid;
    d->sweeps = s->last_sweeps;
    d->noconv = s->noconv;
    d->t_fre = s->t_fre;
    d->V_l0 = s->V_l0;
    return operator_residual(s, &d->op_resid, &d->op_resid_ramp);
}
