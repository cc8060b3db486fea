// lbm_kernels.hpp -- gfx950 kernels of the electrofreezing lattice Boltzmann step.
//
// Layout: every scalar field is one plane of ny rows with a row pitch padded to a
// multiple of 64 elements; a population set is nq consecutive planes ([q][j][i]).
// One thread per node.  Streaming is by pull: the thread of node x fetches
// population q from the source node x - c_q and applies the collision of that
// source node there (the source's collision inputs are read from field planes,
// which neighbouring threads share through the L1/L2 caches).  Each stage reads one
// buffer and writes the other, so the kernels of a stage never race.
//
// Blocks are 256 threads (4 waves of 64) covering a 64 x 4 tile.  The 1-D grid is
// remapped so that each of the 8 XCDs (which receive workgroups round-robin) works
// on one contiguous band of tiles: neighbouring tiles share that XCD's L2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int TX = 64, TY = 4, NT = TX * TY;
constexpr double CS2 = 1.0 / 3.0;
constexpr double W0 = 4.0 / 9.0, WA = 1.0 / 9.0, WD = 1.0 / 36.0;   // D2Q9 weights, Eq. (16)
constexpr double LW0 = 1.0 / 3.0, LWA = 1.0 / 6.0;                  // D2Q5 weights, Eq. (33)

// D2Q9 links in the order rest, E, N, W, S, NE, NW, SW, SE (Eq. (17)).
__device__ constexpr int QX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int QY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int QOPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
__device__ constexpr double QW[9] = {W0, WA, WA, WA, WA, WD, WD, WD, WD};

// Constants of one case, passed by value to every kernel.
struct Dev {
    int nx, ny, pitch;
    int64_t plane;                  // elements per field plane = pitch * ny
    int gx, gy;                     // tiles in x and y
    double omf, facf;               // 1/tau_f and 1 - 1/(2 tau_f)
    double beta, kappa, wet, W;     // Eq. (5) and the wetting slope (4/W) cos(theta)
    double rho_s, rho_l, rho_g, mu_s, mu_l, mu_g;
    double C_s, C_l, C_g, k_s, k_l, k_g;   // volumetric heat capacities, conductivities
    double eps_s, eps_l, eps_g, sig_s, sig_l, sig_g;
    double Cref, Lvol, T_w, T_g;    // C_ref, latent heat per volume, temperatures
    double phi_top, phi_bot, shrink; // shrink = 1 - rho_s / rho_l
    int shape;
    double R0, xc, yc, h0;
    unsigned readings;
};

// Device control block: potential-loop state and step-level reductions.  Reductions use
// no fences or atomics: every block stores its FP64 partial sums, and a later launch (the
// next sweep's block 0, or a one-block finalize kernel) adds them in block order.
struct Ctl {
    int done, count, conv, pad0;     // potential loop: finished, sweeps, converged
    int min_sweeps, max_sweeps;
    double tol, resid;
    double V_l0, V_prev, t_fre;      // freezing-time detector
    long long step;
    int nonfinite, pad1;
    double dsum[6];                  // sum psi, sum f, sum g, V_l, V_s, max |u|
    double front, height;
};

// Offsets into the partial-sum array (nb = blocks of a node-parallel launch).
__host__ __device__ constexpr int64_t part_sweep(int nb, int slot) { return (int64_t)2 * nb * slot; }
__host__ __device__ constexpr int64_t part_vl(int nb) { return (int64_t)4 * nb; }
__host__ __device__ constexpr int64_t part_diag(int nb) { return (int64_t)5 * nb; }
__host__ __device__ constexpr int64_t part_total(int nb) { return (int64_t)12 * nb; }

__device__ __forceinline__ double clamp01(double x) { return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x); }

// Eq. (1) with psi clamped to [0, 1].
__device__ __forceinline__ double mix(double s, double l, double g, double psi, double fs) {
    double pc = clamp01(psi);
    return fs * s + (1.0 - fs) * pc * l + (1.0 - fs) * (1.0 - pc) * g;
}

__device__ __forceinline__ int wrapx(int i, int nx) { return i < 0 ? i + nx : (i >= nx ? i - nx : i); }

__device__ __forceinline__ int64_t at(const Dev& d, int i, int j) { return (int64_t)j * d.pitch + i; }

// Field value with a ghost rule for rows -1 and ny (x already wrapped).
enum Ghost { GMIRROR = 0, GWET = 1, GPHI = 2 };
template <int G>
__device__ __forceinline__ double ghosted(const double* __restrict__ f, const Dev& d, int i, int j) {
    if (j < 0) {
        double b = f[i];
        if (G == GWET) return b + d.wet * b * (1.0 - b);
        if (G == GPHI) return 2.0 * d.phi_bot - b;
        return b;
    }
    if (j >= d.ny) {
        double t = f[at(d, i, d.ny - 1)];
        if (G == GPHI) return 2.0 * d.phi_top - t;
        return t;  // mirror; psi meets the top wall at 90 degrees
    }
    return f[at(d, i, j)];
}

// 3x3 neighbourhood v[dy+1][dx+1] around (i, j).
template <int G>
__device__ __forceinline__ void load3(const double* __restrict__ f, const Dev& d, int i, int j, double v[3][3]) {
    int im = wrapx(i - 1, d.nx), ip = wrapx(i + 1, d.nx);
#pragma unroll
    for (int dy = -1; dy <= 1; dy++) {
        v[dy + 1][0] = ghosted<G>(f, d, im, j + dy);
        v[dy + 1][1] = ghosted<G>(f, d, i, j + dy);
        v[dy + 1][2] = ghosted<G>(f, d, ip, j + dy);
    }
}

// Eq. (36a) and (36b) on a 3x3 neighbourhood.
__device__ __forceinline__ void grad_lap(const double v[3][3], double& gx, double& gy, double& lap) {
    gx = 3.0 * (WA * (v[1][2] - v[1][0]) + WD * (v[2][2] - v[2][0] - v[0][0] + v[0][2]));
    gy = 3.0 * (WA * (v[2][1] - v[0][1]) + WD * (v[2][2] + v[2][0] - v[0][0] - v[0][2]));
    double c = v[1][1];
    lap = 6.0 * (WA * (v[1][2] + v[1][0] + v[2][1] + v[0][1] - 4.0 * c) +
                 WD * (v[2][2] + v[2][0] + v[0][0] + v[0][2] - 4.0 * c));
}

// Tile of this block, XCD-aware.
__device__ __forceinline__ void node_of(const Dev& d, int& i, int& j) {
    int nb = d.gx * d.gy;
    int b = blockIdx.x;
    int per = nb >> 3;
    int lb = (per << 3) == nb ? (b & 7) * per + (b >> 3) : b;
    int bx = lb % d.gx, by = lb / d.gx;
    i = bx * TX + (threadIdx.x & (TX - 1));
    j = by * TY + (threadIdx.x / TX);
}

// Sum over the block in a fixed order; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; w++) r += sh[w];
    return r;
}
__device__ __forceinline__ double block_max(double v, double* sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; w++) r = fmax(r, sh[w]);
    return r;
}

// ---------------------------------------------------------------------------
// Collision of one population at its source node.

// Phase field, Eqs. (15), (18), (19): A = d/dt(psi u) + c_s^2 lambda n.
__device__ __forceinline__ double coll_f(int q, double fq, double psi, double ux, double uy,
                                         double Ax, double Ay, double md, const Dev& d) {
    double cu = QX[q] * ux + QY[q] * uy;
    double feq = QW[q] * psi * (1.0 + 3.0 * cu);
    double F = QW[q] * (3.0 * (QX[q] * Ax + QY[q] * Ay) + psi * md);
    return fq - d.omf * (fq - feq) + d.facf * F;
}

// Flow, Eqs. (21)-(24).  (Ftx, Fty) = F~, (Gx, Gy) = F + rho f_solid.
struct HIn {
    double p, rho, ux, uy, S, Ftx, Fty, Gx, Gy, om;
};
__device__ __forceinline__ double coll_h(int q, double hq, const HIn& a) {
    double cu = QX[q] * a.ux + QY[q] * a.uy;
    double uu = a.ux * a.ux + a.uy * a.uy;
    double s = QW[q] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    double heq = (q == 0 ? (QW[q] - 1.0) : QW[q]) * 3.0 * a.p + a.rho * s;
    double cF = QX[q] * a.Ftx + QY[q] * a.Fty;
    double uF = a.ux * a.Ftx + a.uy * a.Fty;
    double cG = QX[q] * a.Gx + QY[q] * a.Gy;
    double R = QW[q] * (a.S + 3.0 * cG + 9.0 * (cu * cF - CS2 * uF));
    return hq - a.om * (hq - heq) + (1.0 - 0.5 * a.om) * R;
}

// Enthalpy, Eqs. (28)-(29) with the source weighted by omega_i.
struct GIn {
    double H, T, C, ux, uy, om, Q;
};
__device__ __forceinline__ double coll_g(int q, double gq, const GIn& a, double Cref) {
    double uu = a.ux * a.ux + a.uy * a.uy;
    double geq;
    if (q == 0) {
        geq = a.H - Cref * a.T + W0 * (Cref * a.T - 1.5 * a.C * a.T * uu);
    } else {
        double cu = QX[q] * a.ux + QY[q] * a.uy;
        geq = QW[q] * (Cref * a.T + a.C * a.T * (3.0 * cu + 4.5 * (cu * cu - CS2 * uu)));
    }
    return gq - a.om * (gq - geq) + (1.0 - 0.5 * a.om) * QW[q] * a.Q;
}

// Eq. (7) on the volumetric enthalpy, T_s = T_l = 0, latent heat psi * Lvol.
__device__ __forceinline__ void invert(const Dev& d, double H, double psi, double& T, double& fl) {
    double pc = clamp01(psi);
    double Leff = pc * d.Lvol;
    if (H < 0.0) {
        fl = 0.0;
        T = H / mix(d.C_s, d.C_l, d.C_g, pc, pc);
    } else if (H <= Leff) {
        fl = Leff > 0.0 ? H / Leff : 1.0;
        T = 0.0;
    } else {
        fl = 1.0;
        T = (H - Leff) / mix(d.C_s, d.C_l, d.C_g, pc, 0.0);
    }
}

// ---------------------------------------------------------------------------
// Pointers of one stage.

struct State {
    double* f[2];
    double* h[2];
    double* g[2];
    double* l[2];      // D2Q5 moving links E, N, W, S (the rest population never feeds phi)
    double* psi[2];
    double* ux[2];
    double* uy[2];
    double* p[2];
    double* H[2];
    double* T[2];
    double* fs[2];
    double* md[2];
    double* phi[2];
    double *usx, *usy, *pux, *puy, *Ax, *Ay, *oml, *S, *Fx, *Fy;
    double *rho, *Ftx, *Fty, *Gx, *Gy, *omh, *fl;
    double* partials;  // per-block reduction partials
    Ctl* ctl;
};

// ---------------------------------------------------------------------------
// Initialisation (Algorithm 1, first block): fields, equilibria in buffer 0.

__global__ void __launch_bounds__(NT) k_init(Dev d, State s) {
    int i, j;
    node_of(d, i, j);
    if (i >= d.nx || j >= d.ny) return;
    int64_t n = at(d, i, j);
    double v;
    if (d.shape == 1) {
        v = 0.5 * (1.0 + tanh(2.0 * (d.h0 - 0.5 - j) / d.W));
    } else {
        double dx = i - d.xc;
        dx -= d.nx * floor(dx / d.nx + 0.5);
        double dy = j - d.yc;
        v = 0.5 * (1.0 + tanh(2.0 * (d.R0 - sqrt(dx * dx + dy * dy)) / d.W));
    }
    double pc = clamp01(v);
    double Hn = mix(d.C_s, d.C_l, d.C_g, v, 0.0) * d.T_g + pc * d.Lvol;
    double T, fl;
    invert(d, Hn, v, T, fl);
    double fs = pc * (1.0 - fl);
    double phi0 = d.phi_bot + (d.phi_top - d.phi_bot) * (j + 0.5) / d.ny;
    s.psi[0][n] = v;
    s.ux[0][n] = 0; s.uy[0][n] = 0; s.usx[n] = 0; s.usy[n] = 0; s.p[0][n] = 0;
    s.H[0][n] = Hn; s.T[0][n] = T; s.fs[0][n] = fs; s.md[0][n] = 0; s.fl[n] = fl;
    s.pux[n] = 0; s.puy[n] = 0;
    double rho = mix(d.rho_s, d.rho_l, d.rho_g, v, fs);
    double C = mix(d.C_s, d.C_l, d.C_g, v, fs);
    HIn hin{0, rho, 0, 0, 0, 0, 0, 0, 0, 1.0};
    GIn gin{Hn, T, C, 0, 0, 1.0, 0};
#pragma unroll
    for (int q = 0; q < 9; q++) {
        s.f[0][q * d.plane + n] = QW[q] * v;
        s.h[0][q * d.plane + n] = coll_h(q, 0.0, hin);  // omega = 1 returns h_eq
        s.g[0][q * d.plane + n] = coll_g(q, 0.0, gin, d.Cref);
    }
    double l = LWA * phi0;
#pragma unroll
    for (int q = 0; q < 4; q++) s.l[0][q * d.plane + n] = l;
    s.phi[0][n] = (l + l + l + l) / (1.0 - LW0);
}

// ---------------------------------------------------------------------------
// Stage 1a: A = d/dt(psi u) + c_s^2 lambda n at every node (Eqs. (19), (35)),
// then remember psi^n u^n for the next step.
__global__ void __launch_bounds__(NT) k_f_prep(Dev d, State s, int sp) {
    int i, j;
    node_of(d, i, j);
    if (i >= d.nx || j >= d.ny) return;
    int64_t n = at(d, i, j);
    const double* psi = s.psi[sp];
    double v[3][3];
    load3<GWET>(psi, d, i, j, v);
    double gx, gy, lap;
    grad_lap(v, gx, gy, lap);
    double mag = sqrt(gx * gx + gy * gy);
    double nx = 0.0, ny = 0.0;
    if (mag > 1e-12) {
        nx = gx / mag;
        ny = gy / mag;
    }
    double ps = v[1][1];
    double lam = 4.0 * ps * (1.0 - ps) / d.W;
    double ux = s.ux[sp][n], uy = s.uy[sp][n];
    double px = ps * ux, py = ps * uy;
    s.Ax[n] = (px - s.pux[n]) + CS2 * lam * nx;
    s.Ay[n] = (py - s.puy[n]) + CS2 * lam * ny;
    s.pux[n] = px;
    s.puy[n] = py;
}

// Stage 1b: f pulled and collided at its source, half-way bounce-back at the
// walls; psi^{n+1} = sum f / (1 - mdot/2) (Eq. (20)); 1/tau_l for the sweeps.
__global__ void __launch_bounds__(NT) k_f_stream(Dev d, State s, int sp) {
    int i, j;
    node_of(d, i, j);
    if (i >= d.nx || j >= d.ny) return;
    int64_t n = at(d, i, j);
    const double* fsrc = s.f[sp];
    double* fdst = s.f[sp ^ 1];
    const double* psi = s.psi[sp];
    const double* ux = s.ux[sp];
    const double* uy = s.uy[sp];
    const double* md = s.md[sp];
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < 9; q++) {
        int jj = j - QY[q];
        double val;
        if (jj < 0 || jj >= d.ny) {
            int o = QOPP[q];
            val = coll_f(o, fsrc[o * d.plane + n], psi[n], ux[n], uy[n], s.Ax[n], s.Ay[n], md[n], d);
        } else {
            int64_t m = at(d, wrapx(i - QX[q], d.nx), jj);
            val = coll_f(q, fsrc[q * d.plane + m], psi[m], ux[m], uy[m], s.Ax[m], s.Ay[m], md[m], d);
        }
        fdst[q * d.plane + n] = val;
        sum += val;
    }
    double pn = sum / (1.0 - 0.5 * md[n]);
    s.psi[sp ^ 1][n] = pn;
    double sig = mix(d.sig_s, d.sig_l, d.sig_g, pn, s.fs[sp][n]);
    s.oml[n] = 1.0 / (sig / CS2 + 0.5);
}

// 1/tau_l = 1/(sigma/c_s^2 + 1/2) from the current psi and f_s (Sec. 3.4).
__global__ void __launch_bounds__(NT) k_oml(Dev d, State s, int sp) {
    int i, j;
    node_of(d, i, j);
    if (i >= d.nx || j >= d.ny) return;
    int64_t n = at(d, i, j);
    double sig = mix(d.sig_s, d.sig_l, d.sig_g, s.psi[sp][n], s.fs[sp][n]);
    s.oml[n] = 1.0 / (sig / CS2 + 0.5);
}

// ---------------------------------------------------------------------------
// Convergence test of sweep j, run by one block: adds the block partials of that
// sweep in block order and updates the loop state (thread 0).
__device__ __forceinline__ void sweep_check(const Dev& d, const State& s, int j, double* sh) {
    int nb = d.gx * d.gy;
    const double* pv = s.partials + part_sweep(nb, j & 1);
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nb; k += NT) {
        a += pv[2 * k];
        b += pv[2 * k + 1];
    }
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    if (threadIdx.x == 0) {
        Ctl* c = s.ctl;
        double r = a == 0.0 ? 0.0 : (b > 0.0 ? sqrt(a) / sqrt(b) : INFINITY);
        c->resid = r;
        c->count = j;
        int conv = c->tol >= 0.0 && j >= c->min_sweeps && r <= c->tol;
        c->conv = conv;
        if (conv || j >= c->max_sweeps) c->done = 1;
    }
}

// Potential sweep k of a solve (Eqs. (31)-(34)): D2Q5 links pulled and collided at their
// source, half-way anti-bounce-back at the electrodes, the new phi, and per-block FP64
// partial sums of |phi^k - phi^{k-1}|^2 and |phi^k|^2.  Block 0 also tests sweep k-1,
// whose partials the previous launch stored; when that sweep converged, this launch's
// output (written to the other buffer) is discarded and the state after sweep k-1 stands.
// Launch k = max_sweeps + 1 only tests the last sweep.  `lcur` is the buffer holding the
// state before sweep 1.
__global__ void __launch_bounds__(NT) k_sweep(Dev d, State s, int k, int lcur) {
    __shared__ double sh[NT / 64];
    const Ctl* c = s.ctl;
    if (c->done) return;
    if (k > c->max_sweeps) {
        if (blockIdx.x == 0) sweep_check(d, s, k - 1, sh);
        return;
    }
    int src = (lcur + k - 1) & 1;
    const double* lsrc = s.l[src];
    double* ldst = s.l[src ^ 1];
    const double* phs = s.phi[src];
    double* phd = s.phi[src ^ 1];
    int i, j;
    node_of(d, i, j);
    double d2 = 0.0, p2 = 0.0;
    if (i < d.nx && j < d.ny) {
        int64_t n = at(d, i, j);
        const int64_t P = d.plane;
        int64_t nw = at(d, wrapx(i - 1, d.nx), j), ne = at(d, wrapx(i + 1, d.nx), j);
        // E-moving link from the west neighbour, W-moving from the east neighbour
        double l1 = lsrc[0 * P + nw];
        l1 = l1 - s.oml[nw] * (l1 - LWA * phs[nw]);
        double l3 = lsrc[2 * P + ne];
        l3 = l3 - s.oml[ne] * (l3 - LWA * phs[ne]);
        double l2, l4;
        if (j > 0) {
            int64_t m = n - d.pitch;
            l2 = lsrc[1 * P + m];
            l2 = l2 - s.oml[m] * (l2 - LWA * phs[m]);
        } else {
            double o = lsrc[3 * P + n];
            o = o - s.oml[n] * (o - LWA * phs[n]);
            l2 = -o + 2.0 * LWA * d.phi_bot;
        }
        if (j < d.ny - 1) {
            int64_t m = n + d.pitch;
            l4 = lsrc[3 * P + m];
            l4 = l4 - s.oml[m] * (l4 - LWA * phs[m]);
        } else {
            double o = lsrc[1 * P + n];
            o = o - s.oml[n] * (o - LWA * phs[n]);
            l4 = -o + 2.0 * LWA * d.phi_top;
        }
        ldst[0 * P + n] = l1;
        ldst[1 * P + n] = l2;
        ldst[2 * P + n] = l3;
        ldst[3 * P + n] = l4;
        double ph = (l1 + l2 + l3 + l4) / (1.0 - LW0);
        phd[n] = ph;
        double dd = ph - phs[n];
        d2 = dd * dd;
        p2 = ph * ph;
    }
    double bd = block_sum(d2, sh);
    double bp = block_sum(p2, sh);
    int nb = d.gx * d.gy;
    if (threadIdx.x == 0) {
        double* pw = s.partials + part_sweep(nb, k & 1);
        pw[2 * blockIdx.x] = bd;
        pw[2 * blockIdx.x + 1] = bp;
    }
    if (blockIdx.x == 0 && k >= 2) sweep_check(d, s, k - 1, sh);
}

__global__ void k_ctl_reset(Ctl* c, double tol, int min_sweeps, int max_sweeps) {
    c->done = 0;
    c->count = 0;
    c->conv = 0;
    c->resid = 0.0;
    c->tol = tol;
    c->min_sweeps = min_sweeps;
    c->max_sweeps = max_sweeps;
}

// ---------------------------------------------------------------------------
// Stage 3a: surface tension (Eqs. (3)-(5)) and electric force (Eq. (14)) with
// psi^{n+1}; S = rho mdot + u . grad(rho) (Eq. (24)).
__global__ void __launch_bounds__(NT) k_h_prep1(Dev d, State s, int sp, int lcur) {
    int i, j;
    node_of(d, i, j);
    if (i >= d.nx || j >= d.ny) return;
    int64_t n = at(d, i, j);
    const double* psi = s.psi[sp ^ 1];
    const double* fs = s.fs[sp];
    const double* phi = s.phi[lcur];
    double vp[3][3], vf[3][3], vph[3][3], ve[3][3], vr[3][3];
    load3<GWET>(psi, d, i, j, vp);
    load3<GMIRROR>(fs, d, i, j, vf);
    load3<GPHI>(phi, d, i, j, vph);
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) {
            ve[a][b] = mix(d.eps_s, d.eps_l, d.eps_g, vp[a][b], vf[a][b]);
            vr[a][b] = mix(d.rho_s, d.rho_l, d.rho_g, vp[a][b], vf[a][b]);
        }
    double gx, gy, lap;
    grad_lap(vp, gx, gy, lap);
    double ps = vp[1][1];
    double mu = 4.0 * d.beta * ps * (ps - 1.0) * (ps - 0.5) - d.kappa * lap;
    double Fx = mu * gx, Fy = mu * gy;
    double gpx, gpy, lphi, gex, gey, dum;
    grad_lap(vph, gpx, gpy, lphi);
    grad_lap(ve, gex, gey, dum);
    double eps = ve[1][1];
    double Ex = -gpx, Ey = -gpy;
    double qv = -(gex * gpx + gey * gpy + eps * lphi);
    double E2 = Ex * Ex + Ey * Ey;
    Fx += qv * Ex - 0.5 * E2 * gex;
    Fy += qv * Ey - 0.5 * E2 * gey;
    s.Fx[n] = Fx;
    s.Fy[n] = Fy;
    double grx, gry;
    grad_lap(vr, grx, gry, dum);
    s.S[n] = vr[1][1] * s.md[sp][n] + s.ux[sp][n] * grx + s.uy[sp][n] * gry;
}

// Stage 3b: collision inputs of h: rho, F~, F + rho f_solid, 1/tau_h.
__global__ void __launch_bounds__(NT) k_h_prep2(Dev d, State s, int sp) {
    int i, j;
    node_of(d, i, j);
    if (i >= d.nx || j >= d.ny) return;
    int64_t n = at(d, i, j);
    const double* psi = s.psi[sp ^ 1];
    const double* fs = s.fs[sp];
    double vp[3][3], vf[3][3], vr[3][3], vpr[3][3];
    load3<GWET>(psi, d, i, j, vp);
    load3<GMIRROR>(fs, d, i, j, vf);
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) vr[a][b] = mix(d.rho_s, d.rho_l, d.rho_g, vp[a][b], vf[a][b]);
    load3<GMIRROR>(s.p[sp], d, i, j, vpr);
    double grx, gry, gpx, gpy, gsx = 0.0, gsy = 0.0, dum;
    grad_lap(vr, grx, gry, dum);
    grad_lap(vpr, gpx, gpy, dum);
    if (d.readings & 1u) {
        double vs[3][3];
        load3<GMIRROR>(s.S, d, i, j, vs);
        grad_lap(vs, gsx, gsy, dum);
    }
    double rho = vr[1][1];
    double fsn = vf[1][1];
    double Fx = s.Fx[n], Fy = s.Fy[n];
    s.rho[n] = rho;
    s.Ftx[n] = Fx - gpx + CS2 * grx + CS2 * gsx;
    s.Fty[n] = Fy - gpy + CS2 * gry + CS2 * gsy;
    s.Gx[n] = Fx + rho * (fsn * (0.0 - s.usx[n]));
    s.Gy[n] = Fy + rho * (fsn * (0.0 - s.usy[n]));
    double mu = mix(d.mu_s, d.mu_l, d.mu_g, vp[1][1], fsn);
    s.omh[n] = 1.0 / (mu / (rho * CS2) + 0.5);
}

__device__ __forceinline__ HIn h_inputs(const State& s, int sp, int64_t m) {
    return HIn{s.p[sp][m], s.rho[m], s.ux[sp][m], s.uy[sp][m], s.S[m],
               s.Ftx[m], s.Fty[m], s.Gx[m], s.Gy[m], s.omh[m]};
}

// Stage 3c: h pulled and collided at its source, bounce-back at the walls;
// u* (Eq. (25)), u (Eq. (26) with u_s = 0), p (Eq. (27)).
__global__ void __launch_bounds__(NT) k_h_stream(Dev d, State s, int sp) {
    int i, j;
    node_of(d, i, j);
    if (i >= d.nx || j >= d.ny) return;
    int64_t n = at(d, i, j);
    const double* hsrc = s.h[sp];
    double* hdst = s.h[sp ^ 1];
    HIn self = h_inputs(s, sp, n);
    double sx = 0.0, sy = 0.0, s0 = 0.0;
#pragma unroll
    for (int q = 0; q < 9; q++) {
        int jj = j - QY[q];
        double val;
        if (jj < 0 || jj >= d.ny) {
            int o = QOPP[q];
            val = coll_h(o, hsrc[o * d.plane + n], self);
        } else {
            int64_t m = at(d, wrapx(i - QX[q], d.nx), jj);
            val = coll_h(q, hsrc[q * d.plane + m], h_inputs(s, sp, m));
        }
        hdst[q * d.plane + n] = val;
        sx += QX[q] * val;
        sy += QY[q] * val;
        if (q) s0 += val;
    }
    double rho = self.rho;
    double fsn = s.fs[sp][n];
    double ax = (sx + 0.5 * s.Fx[n]) / rho;
    double ay = (sy + 0.5 * s.Fy[n]) / rho;
    s.usx[n] = ax;
    s.usy[n] = ay;
    double ux = ax + 0.5 * fsn * (0.0 - ax);
    double uy = ay + 0.5 * fsn * (0.0 - ay);
    s.ux[sp ^ 1][n] = ux;
    s.uy[sp ^ 1][n] = uy;
    double uF = self.ux * self.Ftx + self.uy * self.Fty;
    double R0 = W0 * (self.S - 3.0 * uF);
    double uu = ux * ux + uy * uy;
    double s0u = W0 * (-1.5 * uu);
    s.p[sp ^ 1][n] = CS2 / (1.0 - W0) * (s0 + 0.5 * self.S + (1.0 / self.om) * R0 + rho * s0u);
}

__device__ __forceinline__ GIn g_inputs(const Dev& d, const State& s, int sp, int64_t m) {
    double ps = s.psi[sp ^ 1][m];
    double fsn = s.fs[sp][m];
    double C = mix(d.C_s, d.C_l, d.C_g, ps, fsn);
    double k = mix(d.k_s, d.k_l, d.k_g, ps, fsn);
    double T = s.T[sp][m];
    return GIn{s.H[sp][m], T, C, s.ux[sp ^ 1][m], s.uy[sp ^ 1][m],
               1.0 / (k / (d.Cref * CS2) + 0.5), C * T * s.md[sp][m]};
}

// Stage 4: g pulled and collided at its source; substrate anti-bounce-back at T_w,
// adiabatic top; H^{n+1} = sum g + Q/2 (Eq. (30)); Eq. (7) gives T, f_l; new f_s
// and mdot.  The FP64 liquid volume feeds the on-device freezing-time detector.
__global__ void __launch_bounds__(NT) k_g_stream(Dev d, State s, int sp) {
    int i, j;
    node_of(d, i, j);
    double vl = 0.0;
    if (i < d.nx && j < d.ny) {
        int64_t n = at(d, i, j);
        const double* gsrc = s.g[sp];
        double* gdst = s.g[sp ^ 1];
        GIn self = g_inputs(d, s, sp, n);
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < 9; q++) {
            int jj = j - QY[q];
            int o = QOPP[q];
            double val;
            if (jj < 0) {
                val = -coll_g(o, gsrc[o * d.plane + n], self, d.Cref) + 2.0 * QW[q] * d.Cref * d.T_w;
            } else if (jj >= d.ny) {
                val = coll_g(o, gsrc[o * d.plane + n], self, d.Cref);
            } else {
                int64_t m = at(d, wrapx(i - QX[q], d.nx), jj);
                val = coll_g(q, gsrc[q * d.plane + m], g_inputs(d, s, sp, m), d.Cref);
            }
            gdst[q * d.plane + n] = val;
            sum += val;
        }
        double Hn = sum + 0.5 * self.Q;
        double ps = s.psi[sp ^ 1][n];
        double T, fl;
        invert(d, Hn, ps, T, fl);
        double fsn = clamp01(ps) * (1.0 - fl);
        s.H[sp ^ 1][n] = Hn;
        s.T[sp ^ 1][n] = T;
        s.fl[n] = fl;
        s.md[sp ^ 1][n] = d.shrink * (fsn - s.fs[sp][n]);
        s.fs[sp ^ 1][n] = fsn;
        vl = clamp01(ps) * fl;
    }
    __shared__ double sh[NT / 64];
    double bv = block_sum(vl, sh);
    if (threadIdx.x == 0) s.partials[part_vl(d.gx * d.gy) + blockIdx.x] = bv;
}

// One block: liquid volume of the new state (block partials in order).  mode 1 records
// V_l0 after initialisation; mode 0 advances the step counter and runs the freezing-time
// detector: t_fre is the first step with V_l <= 1% of V_l0, interpolated linearly.
__global__ void __launch_bounds__(NT) k_vl_finalize(Dev d, State s, int mode) {
    __shared__ double sh[NT / 64];
    int nb = d.gx * d.gy;
    const double* pv = s.partials + part_vl(nb);
    double a = 0.0;
    for (int k = threadIdx.x; k < nb; k += NT) a += pv[k];
    a = block_sum(a, sh);
    if (threadIdx.x != 0) return;
    Ctl* c = s.ctl;
    if (mode == 1) {
        c->V_l0 = a;
        c->V_prev = a;
        c->t_fre = -1.0;
        c->step = 0;
        return;
    }
    long long st = c->step + 1;
    c->step = st;
    double thr = 0.01 * c->V_l0;
    if (c->t_fre < 0.0 && c->V_l0 > 0.0 && a <= thr) {
        double dv = c->V_prev - a;
        c->t_fre = (double)(st - 1) + (dv > 0.0 ? (c->V_prev - thr) / dv : 1.0);
    }
    c->V_prev = a;
}

// Per-block liquid volume of the initial state (finalized by k_vl_finalize, mode 1).
__global__ void __launch_bounds__(NT) k_vl0(Dev d, State s) {
    int i, j;
    node_of(d, i, j);
    double vl = 0.0;
    if (i < d.nx && j < d.ny) {
        int64_t n = at(d, i, j);
        vl = clamp01(s.psi[0][n]) * s.fl[n];
    }
    __shared__ double sh[NT / 64];
    double bv = block_sum(vl, sh);
    if (threadIdx.x == 0) s.partials[part_vl(d.gx * d.gy) + blockIdx.x] = bv;
}

// ---------------------------------------------------------------------------
// Diagnostics: per-block FP64 sums, max |u| and a non-finite count; k_diag_finalize
// adds them in block order and scans the centre column for the droplet height
// (psi = 1/2) and the freezing front (f_l = 1/2).
__global__ void __launch_bounds__(NT) k_diag(Dev d, State s, int sp, int lcur) {
    int i, j;
    node_of(d, i, j);
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    if (i < d.nx && j < d.ny) {
        int64_t n = at(d, i, j);
        double ps = s.psi[sp][n];
        double fl = s.fl[n];
        double ux = s.ux[sp][n], uy = s.uy[sp][n];
        v[0] = ps;
        double sf = 0.0, sg = 0.0;
        for (int q = 0; q < 9; q++) {
            sf += s.f[sp][q * d.plane + n];
            sg += s.g[sp][q * d.plane + n];
        }
        v[1] = sf;
        v[2] = sg;
        v[3] = clamp01(ps) * fl;
        v[4] = s.fs[sp][n];
        v[5] = sqrt(ux * ux + uy * uy);
        double chk = ps + ux + uy + s.p[sp][n] + s.T[sp][n] + s.phi[lcur][n];
        v[6] = isfinite(chk) ? 0.0 : 1.0;
    }
    __shared__ double sh[NT / 64];
    double r[7];
    for (int k = 0; k < 5; k++) r[k] = block_sum(v[k], sh);
    r[5] = block_max(v[5], sh);
    r[6] = block_sum(v[6], sh);
    if (threadIdx.x == 0) {
        double* pw = s.partials + part_diag(d.gx * d.gy) + 7 * (int64_t)blockIdx.x;
        for (int k = 0; k < 7; k++) pw[k] = r[k];
    }
}

__global__ void __launch_bounds__(NT) k_diag_finalize(Dev d, State s, int sp) {
    __shared__ double sh[NT / 64];
    int nb = d.gx * d.gy;
    const double* pv = s.partials + part_diag(nb);
    double a[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int k = threadIdx.x; k < nb; k += NT) {
        for (int m = 0; m < 5; m++) a[m] += pv[7 * k + m];
        a[5] = fmax(a[5], pv[7 * k + 5]);
        a[6] += pv[7 * k + 6];
    }
    double out[7];
    for (int m = 0; m < 5; m++) out[m] = block_sum(a[m], sh);
    out[5] = block_max(a[5], sh);
    out[6] = block_sum(a[6], sh);
    if (threadIdx.x != 0) return;
    Ctl* c = s.ctl;
    for (int m = 0; m < 6; m++) c->dsum[m] = out[m];
    c->nonfinite = out[6] > 0.0;
    const double* psi = s.psi[sp];
    int ic = d.nx / 2;
    double height = 0.0;
    for (int jj = d.ny - 1; jj >= 0; jj--) {
        double a0 = psi[at(d, ic, jj)];
        if (a0 >= 0.5) {
            if (jj == d.ny - 1) {
                height = d.ny;
            } else {
                double b0 = psi[at(d, ic, jj + 1)];
                height = jj + (a0 - 0.5) / (a0 - b0) + 0.5;
            }
            break;
        }
    }
    double front = 0.0;
    if (psi[at(d, ic, 0)] >= 0.5) {
        front = height;
        for (int jj = 0; jj < d.ny && psi[at(d, ic, jj)] >= 0.5; jj++) {
            double a0 = s.fl[at(d, ic, jj)];
            if (a0 >= 0.5) {
                if (jj == 0) {
                    front = 0.0;
                } else {
                    double b0 = s.fl[at(d, ic, jj - 1)];
                    front = (jj - 1) + (0.5 - b0) / (a0 - b0) + 0.5;
                }
                break;
            }
        }
    }
    c->height = height;
    c->front = front;
}

// Pitched plane <-> dense FP64 array copies for get/set (device side).
__global__ void k_pack(Dev d, const double* __restrict__ src, double* __restrict__ dst, int planes) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t per = (int64_t)d.nx * d.ny;
    if (k >= per * planes) return;
    int64_t q = k / per, r = k % per;
    int j = (int)(r / d.nx), i = (int)(r % d.nx);
    dst[k] = src[q * d.plane + at(d, i, j)];
}
__global__ void k_unpack(Dev d, const double* __restrict__ src, double* __restrict__ dst, int planes) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t per = (int64_t)d.nx * d.ny;
    if (k >= per * planes) return;
    int64_t q = k / per, r = k % per;
    int j = (int)(r / d.nx), i = (int)(r % d.nx);
    dst[q * d.plane + at(d, i, j)] = src[k];
}

}  // namespace lbm
