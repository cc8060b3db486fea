// lbm_api.hip -- host implementation of the C ABI declared in include/lbm.h.
//
// The library carves every device array out of the caller's workspace, queues
// kernels on the caller's stream and reads back only the few bytes of the control
// block (potential-loop flags, reductions) through pinned host memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_kernels.hpp"

using lbm::Ctl;
using lbm::Dev;
using lbm::NT;
using lbm::State;

struct lbm_handle {
    lbm_params prm;
    Dev dev;
    State st;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    int nb = 0;               // blocks of a node-parallel launch
    int sp = 0;               // which buffer of the double-buffered sets is current
    int lcur = 0;             // which buffer holds the current potential (l, phi)
    long long step = 0;
    std::vector<int> log;     // sweep counts of every potential solve
    int last_sweeps = 0;
    double last_resid = 0.0;
    int noconv = 0;
    int kprev = 0;            // sweeps of the previous solve (first batch size)
    Ctl* hctl = nullptr;      // pinned host mirror of the control block
    std::string err;
};

namespace {

constexpr size_t ALIGN = 256;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int validate(const lbm_params* p) {
    if (!p) return LBM_EINVAL;
    if (p->nx < 2 || p->ny < 3 || (int64_t)p->nx * p->ny > (int64_t)1 << 31) return LBM_EINVAL;
    if (p->precision != LBM_FP64) return LBM_EINVAL;
    if (!(p->W > 0) || !(p->M > 0) || !(p->gamma >= 0)) return LBM_EINVAL;
    if (!(p->rho_l > 0) || !(p->rho_g > 0) || !(p->rho_s > 0)) return LBM_EINVAL;
    if (!(p->mu_l > 0) || !(p->mu_g > 0) || !(p->mu_s > 0)) return LBM_EINVAL;
    if (!(p->cp_l > 0) || !(p->cp_g > 0) || !(p->cp_s > 0)) return LBM_EINVAL;
    if (!(p->k_l > 0) || !(p->k_g > 0) || !(p->k_s > 0)) return LBM_EINVAL;
    if (!(p->sig_l > 0) || !(p->sig_g > 0) || !(p->sig_s > 0)) return LBM_EINVAL;
    if (!(p->latent >= 0) || p->poisson_max_sweeps < 1) return LBM_EINVAL;
    if (p->shape != 0 && p->shape != 1) return LBM_EINVAL;
    return LBM_OK;
}

Dev make_dev(const lbm_params* p) {
    Dev d{};
    d.nx = p->nx;
    d.ny = p->ny;
    d.pitch = (int)round_up((size_t)p->nx, 64);
    d.plane = (int64_t)d.pitch * p->ny;
    d.gx = (p->nx + lbm::TX - 1) / lbm::TX;
    d.gy = (p->ny + lbm::TY - 1) / lbm::TY;
    double tauf = p->M / lbm::CS2 + 0.5;  // Sec. 3.1
    d.omf = 1.0 / tauf;
    d.facf = 1.0 - 0.5 / tauf;
    d.beta = 12.0 * p->gamma / p->W;      // Eq. (5)
    d.kappa = 1.5 * p->gamma * p->W;
    d.W = p->W;
    d.wet = 4.0 / p->W * std::cos(p->theta_deg * M_PI / 180.0);
    d.rho_s = p->rho_s; d.rho_l = p->rho_l; d.rho_g = p->rho_g;
    d.mu_s = p->mu_s; d.mu_l = p->mu_l; d.mu_g = p->mu_g;
    d.C_s = p->rho_s * p->cp_s; d.C_l = p->rho_l * p->cp_l; d.C_g = p->rho_g * p->cp_g;
    d.k_s = p->k_s; d.k_l = p->k_l; d.k_g = p->k_g;
    d.eps_s = p->eps_s; d.eps_l = p->eps_l; d.eps_g = p->eps_g;
    d.sig_s = p->sig_s; d.sig_l = p->sig_l; d.sig_g = p->sig_g;
    d.Cref = 2.0 * d.C_s * d.C_l / (d.C_s + d.C_l);  // Sec. 3.3
    d.Lvol = p->rho_s * p->latent;
    d.T_w = p->T_w; d.T_g = p->T_g;
    d.phi_top = p->phi_top; d.phi_bot = p->phi_bot;
    d.shrink = 1.0 - p->rho_s / p->rho_l;           // Eq. (2b)
    d.shape = p->shape;
    d.R0 = p->R0; d.xc = p->xc; d.yc = p->yc; d.h0 = p->h0;
    d.readings = p->readings;
    return d;
}

// Bump allocator over the workspace; with base == nullptr it only measures.
struct Carver {
    char* base;
    size_t off = 0;
    double* take(size_t ndouble) {
        off = round_up(off, ALIGN);
        double* r = base ? reinterpret_cast<double*>(base + off) : nullptr;
        off += ndouble * sizeof(double);
        return r;
    }
};

size_t carve(const Dev& d, char* base, State* s, int nb) {
    Carver c{base};
    State t{};
    size_t P = (size_t)d.plane;
    for (int b = 0; b < 2; b++) {
        t.f[b] = c.take(9 * P);
        t.h[b] = c.take(9 * P);
        t.g[b] = c.take(9 * P);
        t.l[b] = c.take(4 * P);
        t.psi[b] = c.take(P); t.ux[b] = c.take(P); t.uy[b] = c.take(P); t.p[b] = c.take(P);
        t.H[b] = c.take(P); t.T[b] = c.take(P); t.fs[b] = c.take(P); t.md[b] = c.take(P);
        t.phi[b] = c.take(P);
    }
    double** singles[] = {&t.usx, &t.usy, &t.pux, &t.puy, &t.Ax, &t.Ay, &t.oml, &t.S, &t.Fx,
                          &t.Fy, &t.rho, &t.Ftx, &t.Fty, &t.Gx, &t.Gy, &t.omh, &t.fl};
    for (double** q : singles) *q = c.take(P);
    t.partials = c.take((size_t)lbm::part_total(nb));
    t.ctl = reinterpret_cast<Ctl*>(c.take((sizeof(Ctl) + 7) / 8));
    if (s) *s = t;
    return round_up(c.off, ALIGN);
}

#define HIPCHK(h, x)                                      \
    do {                                                  \
        hipError_t e_ = (x);                              \
        if (e_ != hipSuccess) {                           \
            (h)->err = std::string(#x) + ": " + hipGetErrorString(e_); \
            return LBM_EHIP;                              \
        }                                                 \
    } while (0)

#define LAUNCHCHK(h) HIPCHK(h, hipGetLastError())

__global__ void k_ctl_zero(Ctl* c) { *c = Ctl{}; }

int fetch_ctl(lbm_handle* h) {
    HIPCHK(h, hipMemcpyAsync(h->hctl, h->st.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

// Potential loop: sweep launches go out in batches.  Block 0 of launch k tests sweep
// k - 1; once a test ends the loop every later launch exits at once, so the sweep count
// is exact while the host reads the flag once per batch.  Launch max_sweeps + 1 only
// tests the last sweep.
int run_sweeps(lbm_handle* h, double tol, int min_sweeps, int max_sweeps, int* sweeps, double* resid) {
    lbm::k_ctl_reset<<<1, 1, 0, h->stream>>>(h->st.ctl, tol, min_sweeps, max_sweeps);
    LAUNCHCHK(h);
    int next = 1;
    int batch = std::max(2, h->kprev * 3 / 4 + 1);
    for (;;) {
        int n = std::min(batch, max_sweeps + 2 - next);
        for (int k = next; k < next + n; k++)
            lbm::k_sweep<<<h->nb, NT, 0, h->stream>>>(h->dev, h->st, k, h->lcur);
        LAUNCHCHK(h);
        next += n;
        int rc = fetch_ctl(h);
        if (rc) return rc;
        if (h->hctl->done || next > max_sweeps + 1) break;
        batch = std::min(std::max(batch * 2, 8), 2048);
    }
    int k = h->hctl->count;
    h->lcur = (h->lcur + k) & 1;
    h->kprev = k;
    h->last_sweeps = k;
    h->last_resid = h->hctl->resid;
    h->log.push_back(k);
    if (sweeps) *sweeps = k;
    if (resid) *resid = h->hctl->resid;
    if (tol >= 0 && !h->hctl->conv) return LBM_ENOCONV;
    return LBM_OK;
}

int one_step(lbm_handle* h) {
    const Dev& d = h->dev;
    int sp = h->sp;
    hipStream_t st = h->stream;
    lbm::k_f_prep<<<h->nb, NT, 0, st>>>(d, h->st, sp);
    lbm::k_f_stream<<<h->nb, NT, 0, st>>>(d, h->st, sp);
    LAUNCHCHK(h);
    int rc = run_sweeps(h, h->prm.poisson_tol, 1, h->prm.poisson_max_sweeps, nullptr, nullptr);
    if (rc == LBM_ENOCONV)
        h->noconv++;
    else if (rc)
        return rc;
    lbm::k_h_prep1<<<h->nb, NT, 0, st>>>(d, h->st, sp, h->lcur);
    lbm::k_h_prep2<<<h->nb, NT, 0, st>>>(d, h->st, sp);
    lbm::k_h_stream<<<h->nb, NT, 0, st>>>(d, h->st, sp);
    lbm::k_g_stream<<<h->nb, NT, 0, st>>>(d, h->st, sp);
    lbm::k_vl_finalize<<<1, NT, 0, st>>>(d, h->st, 0);
    LAUNCHCHK(h);
    h->sp ^= 1;
    h->step++;
    return LBM_OK;
}

// Device plane of a field in the current state.
double* field_ptr(lbm_handle* h, int field) {
    State& s = h->st;
    int sp = h->sp;
    switch (field) {
        case LBM_PSI: return s.psi[sp];
        case LBM_UX: return s.ux[sp];
        case LBM_UY: return s.uy[sp];
        case LBM_USX: return s.usx;
        case LBM_USY: return s.usy;
        case LBM_P: return s.p[sp];
        case LBM_T: return s.T[sp];
        case LBM_H: return s.H[sp];
        case LBM_FS: return s.fs[sp];
        case LBM_MDOT: return s.md[sp];
        case LBM_PSIU_X: return s.pux;
        case LBM_PSIU_Y: return s.puy;
        case LBM_PHI: return s.phi[h->lcur];
        case LBM_FL: return s.fl;
        default: return nullptr;
    }
}

double* pop_ptr(lbm_handle* h, int set, int* nq) {
    State& s = h->st;
    switch (set) {
        case LBM_POP_F: *nq = 9; return s.f[h->sp];
        case LBM_POP_H: *nq = 9; return s.h[h->sp];
        case LBM_POP_G: *nq = 9; return s.g[h->sp];
        case LBM_POP_L: *nq = 4; return s.l[h->lcur];
        default: return nullptr;
    }
}

}  // namespace

extern "C" {

int lbm_workspace_bytes(const lbm_params* p, size_t* bytes) {
    int rc = validate(p);
    if (rc) return rc;
    if (!bytes) return LBM_EINVAL;
    Dev d = make_dev(p);
    *bytes = carve(d, nullptr, nullptr, d.gx * d.gy);
    return LBM_OK;
}

int lbm_init(const lbm_params* p, void* workspace, size_t bytes, void* stream, lbm_handle** out) {
    int rc = validate(p);
    if (rc) return rc;
    if (!workspace || !out || ((uintptr_t)workspace % ALIGN) != 0) return LBM_EINVAL;
    Dev d = make_dev(p);
    int nb = d.gx * d.gy;
    size_t need = carve(d, nullptr, nullptr, nb);
    if (bytes < need) return LBM_ESPACE;
    lbm_handle* h = new (std::nothrow) lbm_handle();
    if (!h) return LBM_EINVAL;
    h->prm = *p;
    h->dev = d;
    h->nb = nb;
    h->stream = (hipStream_t)stream;
    h->ws = (char*)workspace;
    h->ws_bytes = bytes;
    carve(d, h->ws, &h->st, nb);
    if (hipHostMalloc((void**)&h->hctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
        delete h;
        return LBM_EHIP;
    }
    std::memset(h->hctl, 0, sizeof(Ctl));
    k_ctl_zero<<<1, 1, 0, h->stream>>>(h->st.ctl);
    lbm::k_init<<<nb, NT, 0, h->stream>>>(d, h->st);
    lbm::k_oml<<<nb, NT, 0, h->stream>>>(d, h->st, 0);
    if (hipGetLastError() != hipSuccess) {
        lbm_destroy(h);
        return LBM_EHIP;
    }
    // first solve from equilibrium populations: the stopping test counts from sweep 2
    rc = run_sweeps(h, p->poisson_tol, 2, p->poisson_max_sweeps, nullptr, nullptr);
    if (rc && rc != LBM_ENOCONV) {
        lbm_destroy(h);
        return rc;
    }
    lbm::k_vl0<<<nb, NT, 0, h->stream>>>(d, h->st);
    lbm::k_vl_finalize<<<1, NT, 0, h->stream>>>(d, h->st, 1);
    if (hipGetLastError() != hipSuccess || fetch_ctl(h) != LBM_OK) {
        lbm_destroy(h);
        return LBM_EHIP;
    }
    *out = h;
    return LBM_OK;
}

int lbm_step(lbm_handle* h, int n) {
    if (!h) return LBM_ESTATE;
    if (n < 0) return LBM_EINVAL;
    for (int k = 0; k < n; k++) {
        int rc = one_step(h);
        if (rc) return rc;
    }
    return LBM_OK;
}

int lbm_solve_potential(lbm_handle* h, double tol, int max_sweeps, int* sweeps, double* resid) {
    if (!h) return LBM_ESTATE;
    if (max_sweeps < 1) return LBM_EINVAL;
    // tau_l follows the current psi and f_s (as the step does after the f stage)
    lbm::k_oml<<<h->nb, NT, 0, h->stream>>>(h->dev, h->st, h->sp);
    LAUNCHCHK(h);
    return run_sweeps(h, tol, 1, max_sweeps, sweeps, resid);
}

int lbm_diagnostics(lbm_handle* h, lbm_diag* out) {
    if (!h) return LBM_ESTATE;
    if (!out) return LBM_EINVAL;
    lbm::k_diag<<<h->nb, NT, 0, h->stream>>>(h->dev, h->st, h->sp, h->lcur);
    lbm::k_diag_finalize<<<1, NT, 0, h->stream>>>(h->dev, h->st, h->sp);
    LAUNCHCHK(h);
    int rc = fetch_ctl(h);
    if (rc) return rc;
    const Ctl& c = *h->hctl;
    std::memset(out, 0, sizeof *out);
    out->step = h->step;
    out->sum_psi = c.dsum[0];
    out->sum_f = c.dsum[1];
    out->sum_g = c.dsum[2];
    out->V_l = c.dsum[3];
    out->V_s = c.dsum[4];
    out->max_u = c.dsum[5];
    out->front_y = c.front;
    out->height = c.height;
    out->resid = h->last_resid;
    out->sweeps = h->last_sweeps;
    out->noconv = h->noconv;
    out->t_fre = c.t_fre;
    out->V_l0 = c.V_l0;
    out->nonfinite = c.nonfinite;
    return c.nonfinite ? LBM_ENONFINITE : LBM_OK;
}

static int copy_planes(lbm_handle* h, double* dev, void* host, int planes, bool to_host) {
    const Dev& d = h->dev;
    size_t w = (size_t)d.nx * sizeof(double);
    size_t dp = (size_t)d.pitch * sizeof(double);
    size_t rows = (size_t)d.ny * planes;
    if (to_host)
        HIPCHK(h, hipMemcpy2DAsync(host, w, dev, dp, w, rows, hipMemcpyDeviceToHost, h->stream));
    else
        HIPCHK(h, hipMemcpy2DAsync(dev, dp, host, w, w, rows, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm_get_field(lbm_handle* h, int field, double* dst) {
    if (!h) return LBM_ESTATE;
    double* p = field_ptr(h, field);
    if (!p || !dst) return LBM_EINVAL;
    return copy_planes(h, p, dst, 1, true);
}

int lbm_set_field(lbm_handle* h, int field, const double* src) {
    if (!h) return LBM_ESTATE;
    double* p = field_ptr(h, field);
    if (!p || !src) return LBM_EINVAL;
    return copy_planes(h, p, const_cast<double*>(src), 1, false);
}

int lbm_get_pop(lbm_handle* h, int set, double* dst) {
    if (!h) return LBM_ESTATE;
    int nq = 0;
    double* p = pop_ptr(h, set, &nq);
    if (!p || !dst) return LBM_EINVAL;
    return copy_planes(h, p, dst, nq, true);
}

int lbm_set_pop(lbm_handle* h, int set, const double* src) {
    if (!h) return LBM_ESTATE;
    int nq = 0;
    double* p = pop_ptr(h, set, &nq);
    if (!p || !src) return LBM_EINVAL;
    return copy_planes(h, p, const_cast<double*>(src), nq, false);
}

int lbm_sweep_log(lbm_handle* h, int* dst, int cap, int* count) {
    if (!h) return LBM_ESTATE;
    int n = (int)h->log.size();
    if (dst)
        for (int k = 0; k < n && k < cap; k++) dst[k] = h->log[k];
    if (count) *count = n;
    return LBM_OK;
}

int lbm_time_sweeps(lbm_handle* h, int n, float* ms) {
    if (!h) return LBM_ESTATE;
    if (n < 1 || !ms) return LBM_EINVAL;
    hipEvent_t a, b;
    HIPCHK(h, hipEventCreate(&a));
    HIPCHK(h, hipEventCreate(&b));
    lbm::k_ctl_reset<<<1, 1, 0, h->stream>>>(h->st.ctl, -1.0, 1, n);
    HIPCHK(h, hipEventRecord(a, h->stream));
    for (int k = 1; k <= n; k++) lbm::k_sweep<<<h->nb, NT, 0, h->stream>>>(h->dev, h->st, k, h->lcur);
    HIPCHK(h, hipEventRecord(b, h->stream));
    LAUNCHCHK(h);
    HIPCHK(h, hipEventSynchronize(b));
    HIPCHK(h, hipEventElapsedTime(ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    h->lcur = (h->lcur + n) & 1;
    return fetch_ctl(h);
}

int lbm_destroy(lbm_handle* h) {
    if (!h) return LBM_OK;
    (void)hipStreamSynchronize(h->stream);
    if (h->hctl) (void)hipHostFree(h->hctl);
    delete h;
    return LBM_OK;
}

const char* lbm_strerror(int code) {
    switch (code) {
        case LBM_OK: return "ok";
        case LBM_EINVAL: return "invalid argument or parameter";
        case LBM_ENOCONV: return "potential sweeps reached the cap before converging";
        case LBM_ENONFINITE: return "non-finite value in the state";
        case LBM_EHIP: return "HIP runtime error";
        case LBM_ESTATE: return "call out of order";
        case LBM_ESPACE: return "workspace too small";
        default: return "unknown error";
    }
}

const char* lbm_last_error(const lbm_handle* h) { return h ? h->err.c_str() : ""; }

}  // extern "C"
