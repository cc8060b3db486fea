// lbm_api.hip -- host implementation of the C ABI declared in include/lbm.h.
//
// The library carves every device array out of the caller's workspace, queues
// kernels on the caller's stream and reads back only the few bytes of the control
// block (potential-loop flags, reductions) through pinned host memory.  Every stage
// exists for R = double (FP64 form) and R = float (FP32 form); the handle holds the
// state of the precision chosen at lbm_init.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <functional>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "lbm.h"
#include "lbm_kernels.hpp"
#include "nn_state.hpp"

using lbm::Ctl;
using lbm::Dev;
using lbm::NT;
using lbm::State;

struct lbm_handle {
    lbm_params prm;
    Dev dev;
    State<double> sd;         // FP64 form
    State<float> sf;          // FP32 form
    int prec = LBM_FP64;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    int nb = 0;               // blocks of a node-parallel launch
    int sp = 0;               // which buffer of the double-buffered sets is current
    int lcur = 0;             // which of the three buffers holds the current potential (l, phi)
    int swm = 8;              // sweeps per blocked launch
    int swv = 4;              // waves per sweep workgroup
    long long step = 0;
    std::vector<int> log;     // sweep counts of every potential solve
    int last_sweeps = 0;
    double last_resid = 0.0;
    int noconv = 0;
    int init_conv = 1;        // the initial potential solve met the stopping rule
    int kprev = 0;            // sweeps of the previous solve (first batch size)
    int lbswap = 0;           // FP32: the carved base sets have traded places (State::lb, lbx)
    lbm_nn* wnn = nullptr;    // warm-start network used before every step's solve (or none)
    int wfactor = 0;
    Ctl* hctl = nullptr;      // pinned host mirror of the control block
    unsigned long long* hword = nullptr;  // pinned coherent words the loop test publishes to
    unsigned seq = 0;         // sequence number of the last published test
    bool resid_stale = false; // last_resid not yet read back from the control block
    bool vl_pending = false;  // the last step's liquid-volume sum not yet folded into the control block
    bool spent = false;       // lbm_time_stages ran: the state is no longer a state of the method
    Ctl* dctl = nullptr;      // device control block
    double* partials = nullptr;
    std::string err;

    template <typename R> State<R>& st();
};
template <> State<double>& lbm_handle::st<double>() { return sd; }
template <> State<float>& lbm_handle::st<float>() { return sf; }

namespace {

constexpr size_t ALIGN = 256;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int validate(const lbm_params* p) {
    if (!p) return LBM_EINVAL;
    if (p->nx < 2 || p->ny < 3 || (int64_t)p->nx * p->ny > (int64_t)1 << 31) return LBM_EINVAL;
    if (p->precision != LBM_FP64 && p->precision != LBM_FP32 && p->precision != LBM_FP32_FP16STORE) return LBM_EINVAL;
    if (!(p->W > 0) || !(p->M > 0) || !(p->gamma >= 0)) return LBM_EINVAL;
    if (!(p->rho_l > 0) || !(p->rho_g > 0) || !(p->rho_s > 0)) return LBM_EINVAL;
    if (!(p->mu_l > 0) || !(p->mu_g > 0) || !(p->mu_s > 0)) return LBM_EINVAL;
    if (!(p->cp_l > 0) || !(p->cp_g > 0) || !(p->cp_s > 0)) return LBM_EINVAL;
    if (!(p->k_l > 0) || !(p->k_g > 0) || !(p->k_s > 0)) return LBM_EINVAL;
    if (!(p->sig_l > 0) || !(p->sig_g > 0) || !(p->sig_s > 0)) return LBM_EINVAL;
    if (!(p->latent >= 0) || p->poisson_max_sweeps < 1) return LBM_EINVAL;
    if (p->shape != 0 && p->shape != 1) return LBM_EINVAL;
    if (p->sweep_block != 0 && p->sweep_block != 1 && p->sweep_block != 2 && p->sweep_block != 4 &&
        p->sweep_block != 8 && p->sweep_block != 16)
        return LBM_EINVAL;
    if (p->sweep_waves != 0 && p->sweep_waves != 4 && p->sweep_waves != 8) return LBM_EINVAL;
    // 16 sweeps shrink a 64-row tile to 32 written rows; a 32-row tile would write none
    if (p->sweep_block == 16 && p->sweep_waves != 8) return LBM_EINVAL;
    if (p->skip_initial_solve != 0 && p->skip_initial_solve != 1) return LBM_EINVAL;
    if (p->stage_rows < 0 || p->stage_rows > 512 || p->stage_rows % lbm::WR) return LBM_EINVAL;
    return LBM_OK;
}

int sweep_m(const lbm_params* p) { return p->sweep_block ? p->sweep_block : 8; }
int sweep_w(const lbm_params* p) { return p->sweep_waves ? p->sweep_waves : 4; }

// Calls f(M, WV) with the sweep shape as compile-time constants.
template <int M, typename F>
void with_waves(int wv, F&& f) {
    if (wv == 8) f(std::integral_constant<int, M>{}, std::integral_constant<int, 8>{});
    else f(std::integral_constant<int, M>{}, std::integral_constant<int, 4>{});
}
template <typename F>
void with_shape(int m, int wv, F&& f) {
    switch (m) {
        case 1: with_waves<1>(wv, f); break;
        case 2: with_waves<2>(wv, f); break;
        case 4: with_waves<4>(wv, f); break;
        case 16: f(std::integral_constant<int, 16>{}, std::integral_constant<int, 8>{}); break;
        default: with_waves<8>(wv, f); break;
    }
}

Dev make_dev(const lbm_params* p) {
    Dev d{};
    d.nx = p->nx;
    d.ny = p->ny;
    d.pitch = (int)round_up((size_t)p->nx, 64);
    d.plane = (int64_t)d.pitch * p->ny;
    d.gx = (p->nx + lbm::TX - 1) / lbm::TX;
    d.gy = (p->ny + lbm::TY - 1) / lbm::TY;
    int m = sweep_m(p);
    d.tbx = (p->nx + (64 - 2 * m) - 1) / (64 - 2 * m);
    int ry = lbm::SW_NPT * sweep_w(p);
    d.tby = (p->ny + (ry - 2 * m) - 1) / (ry - 2 * m);
    // stage segments: the caller's height, else as tall as 32 rows while the flow launch
    // keeps at least 2048 workgroups
    d.hx = (p->nx + lbm::WX - 1) / lbm::WX;
    d.hseg = p->stage_rows;
    if (d.hseg == 0) {
        d.hseg = 32;
        while (d.hseg > lbm::WR && (int64_t)d.hx * ((p->ny + d.hseg - 1) / d.hseg) < 2048) d.hseg -= lbm::WR;
    }
    d.hy = (p->ny + d.hseg - 1) / d.hseg;
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
    template <typename T>
    T* take(size_t n) {
        off = round_up(off, ALIGN);
        T* r = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += n * sizeof(T);
        return r;
    }
};

// h16: the f, h and g sets in binary16 (the FP16-storage form; R = float).
template <typename R>
size_t carve(const Dev& d, char* base, State<R>* s, bool h16 = false) {
    int nb = lbm::part_nb(d), nbt = d.tbx * d.tby;
    Carver c{base};
    State<R> t{};
    size_t P = (size_t)d.plane;
    for (int b = 0; b < 2; b++) {
        R** sets[] = {&t.f[b], &t.h[b], &t.g[b]};
        for (R** q : sets) *q = h16 ? reinterpret_cast<R*>(c.take<lbm::half_t>(9 * P)) : c.take<R>(9 * P);
        t.psi[b] = c.take<R>(P); t.ux[b] = c.take<R>(P); t.uy[b] = c.take<R>(P); t.p[b] = c.take<R>(P);
        t.H[b] = c.take<R>(P); t.T[b] = c.take<R>(P); t.fs[b] = c.take<R>(P); t.md[b] = c.take<R>(P);
    }
    for (int b = 0; b < 3; b++) {
        t.l[b] = c.take<R>(4 * P);
        t.phi[b] = c.take<R>(P);
    }
    // the deviation bases exist only in the FP32 form
    const bool based = std::is_same<R, float>::value;
    t.lb = based ? c.take<R>(4 * P) : nullptr;
    t.lbx = based ? c.take<R>(4 * P) : nullptr;
    t.dl = based ? c.take<R>(4 * P) : nullptr;
    t.pbp = based ? c.take<R>(P) : nullptr;
    t.hb = based ? c.take<R>(P) : nullptr;
    R** singles[] = {&t.usx[0], &t.usx[1], &t.usy[0], &t.usy[1], &t.pux, &t.puy, &t.oml, &t.fl};
    for (R** q : singles) *q = c.take<R>(P);
    t.partials = c.take<double>((size_t)lbm::part_alloc(nb, nbt));
    t.ctl = c.take<Ctl>(1);
    if (s) *s = t;
    return round_up(c.off, ALIGN);
}

size_t carve_bytes(const lbm_params* p, const Dev& d) {
    return p->precision == LBM_FP64 ? carve<double>(d, nullptr, nullptr)
                                    : carve<float>(d, nullptr, nullptr, p->precision == LBM_FP32_FP16STORE);
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

// The last step's liquid-volume sum and freezing-time detector are folded into the control
// block by the next step's first kernel; a reader of the control block before that gets them
// from here.
int flush_vl(lbm_handle* h) {
    if (!h->vl_pending) return LBM_OK;
    lbm::k_vl_finalize<<<1, NT, 0, h->stream>>>(h->dev, h->partials, h->dctl, 0, 0);
    LAUNCHCHK(h);
    h->vl_pending = false;
    return LBM_OK;
}

int fetch_ctl(lbm_handle* h) {
    int frc = flush_vl(h);
    if (frc) return frc;
    HIPCHK(h, hipMemcpyAsync(h->hctl, h->dctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (h->resid_stale) {
        h->last_resid = h->hctl->resid;
        h->resid_stale = false;
    }
    return LBM_OK;
}

template <typename R, int Tag = 0>
void launch_sweep(lbm_handle* h, const lbm::SweepLaunch& a) {
    int nbt = h->dev.tbx * h->dev.tby;
    State<R>& s = h->st<R>();
    with_shape(h->swm, h->swv, [&](auto M, auto WV) {
        // one block for the test of the previous launch and one per tile
        lbm::k_sweep_tb<M, R, WV, Tag><<<nbt + 1, 64 * WV, 0, h->stream>>>(h->dev, s, a);
    });
}

template <typename R>
void launch_test(lbm_handle* h, const lbm::SweepLaunch& a, unsigned seq, bool publish = true) {
    State<R>& s = h->st<R>();
    unsigned long long* w = publish ? h->hword : nullptr;
    // range sums in parallel when there are enough tiles to share out
    const int nbt = h->dev.tbx * h->dev.tby;
    const int parts = std::min(lbm::TEST_RANGES, nbt / lbm::TEST_NT);
    with_shape(h->swm, 4, [&](auto M, auto) {
        if (parts > 1)
            lbm::k_sweep_test_part<M(), R><<<parts, lbm::TEST_NT, 0, h->stream>>>(h->dev, s, a);
        lbm::k_sweep_test<M(), R><<<1, lbm::TEST_NT, 0, h->stream>>>(h->dev, s, a, parts > 1 ? parts : 0, w, seq);
    });
}

// Outcome of a loop test as published by k_sweep_test.
struct LoopState {
    int done, conv, count, fix_launch, fix_n;
};

// Wait for the test with sequence number `seq`: spin on the two published words (the GPU
// keeps running the queued work meanwhile); after 2 s without them, synchronise the stream
// (which reports a failed launch) and look once more.
int wait_test(lbm_handle* h, unsigned seq, LoopState* out) {
    auto ready = [&](unsigned long long& w0, unsigned long long& w1) {
        w0 = __atomic_load_n(&h->hword[0], __ATOMIC_ACQUIRE);
        w1 = __atomic_load_n(&h->hword[1], __ATOMIC_ACQUIRE);
        return (unsigned)(w0 >> 32) == seq && (unsigned)(w1 >> 32) == seq;
    };
    unsigned long long w0 = 0, w1 = 0;
    auto t0 = std::chrono::steady_clock::now();
    while (!ready(w0, w1)) {
        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
            HIPCHK(h, hipStreamSynchronize(h->stream));
            if (ready(w0, w1)) break;
            h->err = "potential loop test was not published";
            return LBM_EHIP;
        }
    }
    out->count = (int)(unsigned)w0;
    const unsigned b = (unsigned)w1;
    out->done = b & 1u;
    out->conv = (b >> 1) & 1u;
    out->fix_n = (b >> 2) & 31u;  // up to 16
    out->fix_launch = (int)(b >> 7);
    return LBM_OK;
}

// Potential loop.  Sweeps go out in blocked launches of up to swm sweeps; an extra block of
// each launch tests every sweep of the previous launch, and each batch of launches ends
// with a one-block test of its last launch, after which the host reads the outcome.  The
// first batch covers the previous solve's count, later batches double from one sweep.
// Launches queued after a test ended the loop exit at once.  If the final sweep is not
// the last of its launch, that launch's sweeps up to it are recomputed from its input
// (three buffers keep that input intact past the launches that follow it in the batch,
// which all exit at once): by the host after it read the outcome, or, with `tail` (the
// rest of a time step), on the device, queued with the tail behind every batch's test.
template <typename R>
int run_sweeps(lbm_handle* h, double tol, int min_sweeps, int max_sweeps, int* sweeps, double* resid,
               bool armed = false, const std::function<void()>* tail = nullptr) {
    if (std::is_same<R, float>::value) {
        // renormalised pairs into the next potential buffer and the other base set
        State<R>& s = h->st<R>();
        const int lnew = (h->lcur + 1) % 3;
        lbm::k_rebase_prep<R><<<h->nb, NT, 0, h->stream>>>(h->dev, s, h->lcur, lnew);
        std::swap(s.lb, s.lbx);
        h->lbswap ^= 1;
        h->lcur = lnew;
    }
    // armed: an earlier kernel of the step already reset the loop with these tol/min/max
    if (!armed) lbm::k_ctl_reset<<<1, 1, 0, h->stream>>>(h->dctl, tol, min_sweeps, max_sweeps);
    LAUNCHCHK(h);
    std::vector<lbm::SweepLaunch> plan;
    LoopState ls{};
    int next = 1;       // next sweep index
    int buf = h->lcur;  // buffer holding the state before sweep `next`
    const int lcur0 = h->lcur;
    // Sweeps per batch.  A launch costs little more than the traffic of its first sweep (one
    // read and one write of the links, halo included), so the plan avoids launches rather than
    // sweeps that run in vain: the first batch covers exactly the previous solve's count,
    // which changes by a sweep or two from one time step to the next.  A stop before the end
    // of the batch's last launch costs the recomputation of the stopping launch (the lagged
    // test in the launch after it sees a stop earlier in the batch); a solve that needs more
    // costs a host round trip and a short launch: later batches double from one sweep.  A
    // batch goes out as launches of up to swm sweeps; none straddles an FP32 rebase point.
    const long long most = 256LL * h->swm;
    long long budget = h->kprev > 0 ? std::min<long long>(h->kprev, most) : h->swm;
    long long grow = 1;
    const bool rebasing = std::is_same<R, float>::value;
    for (;;) {
        for (int c = 0; budget > 0 && next <= max_sweeps; c++) {
            // FP32 rebase points (every REBASE_SWEEPS sweeps, whatever the launch sizes):
            // inside a batch, the launch just queued is tested first (nothing published) and
            // the renormalisation and its constants run only if the loop goes on, so a rebase
            // costs no host round trip; at the start of a later batch the loop is known to go on
            if (rebasing && next > 1 && (next - 1) % lbm::REBASE_SWEEPS == 0) {
                if (c > 0) {
                    const lbm::SweepLaunch& last = plan.back();
                    lbm::SweepLaunch mid{};
                    mid.prev_k0 = last.k0;
                    mid.prev_nsw = last.nsw;
                    mid.prev_slot = last.slot;
                    mid.launch = (int)plan.size();
                    mid.src = lcur0;
                    launch_test<R>(h, mid, 0, false);
                }
                lbm::k_rebase<R><<<h->nb, NT, 0, h->stream>>>(h->dev, h->st<R>(), buf, 1);
                lbm::k_sweep_prep<R><<<h->nb, NT, 0, h->stream>>>(h->dev, h->st<R>(), 1);
            }
            lbm::SweepLaunch a{};
            int t = (int)plan.size();
            int nsw = (int)std::min<long long>(std::min<long long>(h->swm, budget), max_sweeps + 1 - next);
            if (rebasing) nsw = std::min(nsw, lbm::REBASE_SWEEPS - (next - 1) % lbm::REBASE_SWEEPS);
            a.nsw = nsw;
            a.src = buf;
            a.dst = (buf + 1) % 3;
            a.k0 = next;
            a.slot = t & 1;
            a.launch = t;
            if (t > 0) {
                a.prev_k0 = plan[t - 1].k0;
                a.prev_nsw = plan[t - 1].nsw;
                a.prev_slot = plan[t - 1].slot;
            }
            launch_sweep<R>(h, a);
            plan.push_back(a);
            next += nsw;
            budget -= nsw;
            buf = a.dst;
        }
        lbm::SweepLaunch tst{};
        const lbm::SweepLaunch& last = plan.back();
        tst.prev_k0 = last.k0;
        tst.prev_nsw = last.nsw;
        tst.prev_slot = last.slot;
        tst.launch = (int)plan.size();
        tst.src = lcur0;
        const unsigned seq = ++h->seq;
        launch_test<R>(h, tst, seq);
        if (tail) {
            // what follows the loop goes out before the host reads the outcome: the
            // recomputation of the stopping launch and the gated stage kernels run only if
            // this test (or an earlier one) ended the loop, so the device does not wait for
            // the host round trip
            lbm::SweepLaunch fx{};
            fx.devfix = 1;
            fx.src = lcur0;
            launch_sweep<R>(h, fx);
            (*tail)();
        }
        LAUNCHCHK(h);
        int rc = wait_test(h, seq, &ls);
        if (rc) return rc;
        if (ls.done || next > max_sweeps) break;
        budget = grow;
        grow = std::min(grow * 2, most);
    }
    if (!ls.done) {
        h->err = "potential loop ended without a decision";
        return LBM_EHIP;
    }
    int k = ls.count;
    const lbm::SweepLaunch& f = plan[ls.fix_launch];
    int final_buf = f.dst;
    if (ls.fix_n != f.nsw && tail) {
        final_buf = (f.src + 2) % 3;  // recomputed on the device (devfix) behind the last test
    } else if (ls.fix_n != f.nsw) {
        lbm::SweepLaunch a{};
        a.src = f.src;
        a.dst = (f.src + 2) % 3;
        a.nsw = ls.fix_n;
        a.k0 = f.k0;
        a.slot = (int)plan.size() & 1;
        a.launch = (int)plan.size();
        a.force = 1;
        launch_sweep<R>(h, a);
        LAUNCHCHK(h);
        final_buf = a.dst;
    }
    h->lcur = final_buf;
    h->kprev = k;
    h->last_sweeps = k;
    h->resid_stale = true;  // the final residual stays on the device until someone asks
    h->log.push_back(k);
    if (sweeps) *sweeps = k;
    if (resid) {
        int rc = fetch_ctl(h);
        if (rc) return rc;
        *resid = h->hctl->resid;
    }
    if (tol >= 0 && !ls.conv) return LBM_ENOCONV;
    return LBM_OK;
}

template <typename R, bool H = false>
int one_step(lbm_handle* h) {
    const Dev& d = h->dev;
    int sp = h->sp;
    hipStream_t st = h->stream;
    State<R>& s = h->st<R>();
    const double tol = h->prm.poisson_tol;
    const int maxsw = h->prm.poisson_max_sweeps;
    const int fin = h->vl_pending ? 1 : 0;
    lbm::k_f_fused_arm<R, H><<<d.gx * d.hy + fin, NT, 0, st>>>(d, s, sp, tol, 1, maxsw, fin);
    h->vl_pending = false;
    LAUNCHCHK(h);
    if (h->wnn) {
        // warm start from the network: maps of the new psi (and f_s^n, as 1/tau_l uses)
        const int f = h->wfactor, nxc = d.nx / f, nyc = d.ny / f;
        lbm::k_nn_features<R><<<(nxc * nyc + NT - 1) / NT, NT, 0, st>>>(d, s, sp ^ 1, sp, f, h->wnn->x);
        LAUNCHCHK(h);
        int frc = nnapi::forward(h->wnn, h->wnn->x, h->wnn->y, 1, nyc, nxc, st);
        if (frc) {
            h->err = h->wnn->err;
            return frc;
        }
        lbm::k_nn_seed<R><<<h->nb, NT, 0, st>>>(d, s, h->lcur, f, h->wnn->y);
        LAUNCHCHK(h);
    }
    // stages 3-4 and the volume sum, gated on the loop's end and reading its final buffer
    // from the control block; queued behind every test of the loop (see run_sweeps)
    const std::function<void()> tail = [&]() {
        lbm::k_h_fused<R, H><<<d.hx * d.hy, NT, 0, st>>>(d, s, sp, -1);
        lbm::k_g_stream<R, H><<<d.gx * d.hy, NT, 0, st>>>(d, s, sp, 1);
    };
    int rc = run_sweeps<R>(h, tol, 1, maxsw, nullptr, nullptr, true, &tail);
    if (rc == LBM_ENOCONV)
        h->noconv++;
    else if (rc)
        return rc;
    LAUNCHCHK(h);
    h->vl_pending = true;
    h->sp ^= 1;
    h->step++;
    return LBM_OK;
}

template <typename R, bool H = false>
int init_state(lbm_handle* h) {
    const Dev& d = h->dev;
    State<R>& s = h->st<R>();
    k_ctl_zero<<<1, 1, 0, h->stream>>>(h->dctl);
    lbm::k_init<R, H><<<h->nb, NT, 0, h->stream>>>(d, s);
    lbm::k_oml<R><<<h->nb, NT, 0, h->stream>>>(d, s, 0);
    LAUNCHCHK(h);
    int solve_rc = LBM_OK;
    if (h->prm.skip_initial_solve) {
        // the caller seeds and solves the potential (warm start); the ramp stays for now
        h->log.push_back(0);
    } else {
        // first solve from equilibrium populations: the stopping test counts from sweep 2
        solve_rc = run_sweeps<R>(h, h->prm.poisson_tol, 2, h->prm.poisson_max_sweeps, nullptr, nullptr);
        if (solve_rc && solve_rc != LBM_ENOCONV) return solve_rc;
        h->init_conv = solve_rc == LBM_OK;
    }
    lbm::k_vl0<R><<<d.gx * d.hy, NT, 0, h->stream>>>(d, s);
    lbm::k_vl_finalize<<<1, NT, 0, h->stream>>>(d, h->partials, h->dctl, 1, 0);
    LAUNCHCHK(h);
    int rc = fetch_ctl(h);
    return rc ? rc : solve_rc;
}

template <typename R>
int solve_potential(lbm_handle* h, double tol, int max_sweeps, int* sweeps, double* resid) {
    // tau_l follows the current psi and f_s (as the step does after the f stage)
    lbm::k_oml<R><<<h->nb, NT, 0, h->stream>>>(h->dev, h->st<R>(), h->sp);
    LAUNCHCHK(h);
    return run_sweeps<R>(h, tol, 1, max_sweeps, sweeps, resid);
}

template <typename R, bool H = false>
int diagnostics(lbm_handle* h) {
    int frc = flush_vl(h);
    if (frc) return frc;
    lbm::k_diag<R, H><<<h->nb, NT, 0, h->stream>>>(h->dev, h->st<R>(), h->sp, h->lcur);
    lbm::k_diag_finalize<R><<<1, NT, 0, h->stream>>>(h->dev, h->st<R>(), h->sp);
    LAUNCHCHK(h);
    return fetch_ctl(h);
}

template <typename R, int Tag>
int time_sweeps(lbm_handle* h, int n, float* ms) {
    hipEvent_t a, b;
    HIPCHK(h, hipEventCreate(&a));
    HIPCHK(h, hipEventCreate(&b));
    if (std::is_same<R, float>::value) {
        lbm::k_rebase<R><<<h->nb, NT, 0, h->stream>>>(h->dev, h->st<R>(), h->lcur, 0);
        lbm::k_sweep_prep<R><<<h->nb, NT, 0, h->stream>>>(h->dev, h->st<R>(), 0);
    }
    lbm::k_ctl_reset<<<1, 1, 0, h->stream>>>(h->dctl, -1.0, 1, n);
    HIPCHK(h, hipEventRecord(a, h->stream));
    int buf = h->lcur;
    lbm::SweepLaunch prev{};
    for (int k = 1, t = 0; k <= n; t++) {
        // as in a solve: block 0 also tests the previous launch (never converging here)
        lbm::SweepLaunch s{};
        s.nsw = std::min(h->swm, n + 1 - k);
        s.src = buf;
        s.dst = (buf + 1) % 3;
        s.k0 = k;
        s.slot = t & 1;
        s.launch = t;
        if (t > 0) {
            s.prev_k0 = prev.k0;
            s.prev_nsw = prev.nsw;
            s.prev_slot = prev.slot;
        }
        launch_sweep<R, Tag>(h, s);
        prev = s;
        buf = s.dst;
        k += s.nsw;
    }
    HIPCHK(h, hipEventRecord(b, h->stream));
    LAUNCHCHK(h);
    HIPCHK(h, hipEventSynchronize(b));
    HIPCHK(h, hipEventElapsedTime(ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    h->lcur = buf;
    return fetch_ctl(h);
}

// Measurement: each stage kernel of the step launched n times back to back on the current
// state, bracketed by HIP events (each reads buffer sp and writes the other, so a repeat
// rewrites the same values).  The kernels are the step's own, ungated.
constexpr int NSTAGES = 3;
const char* const STAGE_NAMES[NSTAGES] = {"k_f_fused_arm", "k_h_fused", "k_g_stream"};

template <typename R, bool H = false>
int time_stages(lbm_handle* h, int n, float* ms) {
    const Dev& d = h->dev;
    State<R>& s = h->st<R>();
    const int sp = h->sp;
    hipStream_t st = h->stream;
    int frc = flush_vl(h);  // the f kernel's extra block would fold a pending volume sum
    if (frc) return frc;
    hipEvent_t ev[NSTAGES + 1];
    for (auto& e : ev) HIPCHK(h, hipEventCreate(&e));
    HIPCHK(h, hipEventRecord(ev[0], st));
    for (int k = 0; k < n; k++)
        lbm::k_f_fused_arm<R, H><<<d.gx * d.hy, NT, 0, st>>>(d, s, sp, h->prm.poisson_tol, 1, h->prm.poisson_max_sweeps, 0);
    HIPCHK(h, hipEventRecord(ev[1], st));
    for (int k = 0; k < n; k++) lbm::k_h_fused<R, H><<<d.hx * d.hy, NT, 0, st>>>(d, s, sp, h->lcur);
    HIPCHK(h, hipEventRecord(ev[2], st));
    for (int k = 0; k < n; k++) lbm::k_g_stream<R, H><<<d.gx * d.hy, NT, 0, st>>>(d, s, sp, 0);
    HIPCHK(h, hipEventRecord(ev[3], st));
    LAUNCHCHK(h);
    HIPCHK(h, hipEventSynchronize(ev[NSTAGES]));
    for (int k = 0; k < NSTAGES; k++) {
        float t = 0.f;
        HIPCHK(h, hipEventElapsedTime(&t, ev[k], ev[k + 1]));
        ms[k] = t / (float)n;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    return LBM_OK;
}

// Device plane(s) of a field or population set in the current state, with the offset
// kind that converts stored values to the raw FP64 values of the ABI.
// enthalpy base; potential link bases; FP32 phase-field populations held as deviations from
// w_i psi of their node
enum Offset { OFF_NONE, OFF_G, OFF_BASE, OFF_F };

template <typename R>
R* field_ptr(lbm_handle* h, int field, Offset* off) {
    State<R>& s = h->st<R>();
    int sp = h->sp;
    *off = OFF_NONE;
    switch (field) {
        case LBM_PSI: return s.psi[sp];
        case LBM_UX: return s.ux[sp];
        case LBM_UY: return s.uy[sp];
        case LBM_USX: return s.usx[sp];
        case LBM_USY: return s.usy[sp];
        case LBM_P: return s.p[sp];
        case LBM_T: return s.T[sp];
        case LBM_H: *off = h->prec != LBM_FP64 ? OFF_G : OFF_NONE; return s.H[sp];
        case LBM_FS: return s.fs[sp];
        case LBM_MDOT: return s.md[sp];
        case LBM_PSIU_X: return s.pux;
        case LBM_PSIU_Y: return s.puy;
        case LBM_PHI: return s.phi[h->lcur];
        case LBM_FL: return s.fl;
        default: return nullptr;
    }
}

template <typename R>
R* pop_ptr(lbm_handle* h, int set, int* nq, Offset* off) {
    State<R>& s = h->st<R>();
    *off = OFF_NONE;
    switch (set) {
        case LBM_POP_F: *nq = 9; *off = h->prec != LBM_FP64 ? OFF_F : OFF_NONE; return s.f[h->sp];
        case LBM_POP_H: *nq = 9; return s.h[h->sp];
        case LBM_POP_G: *nq = 9; *off = h->prec != LBM_FP64 ? OFF_G : OFF_NONE; return s.g[h->sp];
        case LBM_POP_L: *nq = 4; *off = h->prec != LBM_FP64 ? OFF_BASE : OFF_NONE; return s.l[h->lcur];
        default: return nullptr;
    }
}

// Offset added to stored values of plane q to give raw values (base: per node).
// Host copies of pitched planes go through one contiguous block (rows x pitch elements, the
// planes follow each other without gaps): the stream is drained, then a blocking 1-D copy.
// (Pitched 2-D copies returned zeros while a kernel tracer was attached.)
template <typename R>
int block_to_host(lbm_handle* h, std::vector<R>& blk, const R* dev, size_t elems) {
    blk.resize(elems);
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(blk.data(), dev, elems * sizeof(R), hipMemcpyDeviceToHost));
    return LBM_OK;
}
template <typename R>
int block_to_dev(lbm_handle* h, R* dev, const std::vector<R>& blk) {
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(dev, blk.data(), blk.size() * sizeof(R), hipMemcpyHostToDevice));
    return LBM_OK;
}

template <typename R>
int copy_planes(lbm_handle* h, R* dev, double* host, int planes, bool to_host, Offset off) {
    const Dev& d = h->dev;
    const size_t nx = (size_t)d.nx, pitch = (size_t)d.pitch, ny = (size_t)d.ny;
    const size_t per = nx * ny;
    // OFF_G: one enthalpy base plane (applies to H and to the rest link of g);
    // OFF_BASE: one base plane per potential link
    std::vector<R> base;
    const size_t bplanes = off == OFF_BASE ? (size_t)planes : 1;
    R* bp = off == OFF_BASE ? h->st<R>().lb : (off == OFF_F ? h->st<R>().psi[h->sp] : h->st<R>().hb);
    if (off == OFF_G || off == OFF_F || (off == OFF_BASE && to_host)) {
        int rc = block_to_host<R>(h, base, bp, ny * pitch * bplanes);
        if (rc) return rc;
    }
    // element k = (plane, j, i) of the host array -> pitched index
    auto pidx = [&](size_t k) { return (k / nx) * pitch + k % nx; };
    auto offset = [&](size_t k) -> double {
        if (off == OFF_G) return (planes == 1 || k < per) ? (double)base[pidx(k % per)] : 0.0;
        if (off == OFF_BASE) return (double)base[pidx(k)];
        if (off == OFF_F) {  // w_i psi as the kernels form it
            const int q = (int)(k / per);
            const double w = q == 0 ? lbm::W0 : (q < 5 ? lbm::WA : lbm::WD);
            return (double)((R)w * base[pidx(k % per)]);
        }
        return 0.0;
    };
    std::vector<R> blk;
    int rc = block_to_host<R>(h, blk, dev, ny * pitch * planes);
    if (rc) return rc;
    if (to_host) {
        for (size_t k = 0; k < per * planes; k++) host[k] = (double)blk[pidx(k)] + offset(k);
        return LBM_OK;
    }
    if (off == OFF_BASE) {
        // a written link becomes the pair (fl(v), fl(v - fl(v)))
        base.assign(ny * pitch * bplanes, R(0));
        for (size_t k = 0; k < per * planes; k++) base[pidx(k)] = (R)host[k];
        rc = block_to_dev<R>(h, bp, base);
        if (rc) return rc;
    }
    for (size_t k = 0; k < per * planes; k++) blk[pidx(k)] = (R)(host[k] - offset(k));
    return block_to_dev<R>(h, dev, blk);
}

// One field into caller device memory as FP64, row-major without pitch, with the enthalpy
// base added where the FP32 forms keep one (base == nullptr: none).
template <typename R>
__global__ void __launch_bounds__(NT) k_field_out(Dev d, const R* __restrict__ src, const R* __restrict__ base,
                                                  double* __restrict__ dst) {
    const int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (k >= (int64_t)d.nx * d.ny) return;
    const int i = (int)(k % d.nx), j = (int)(k / d.nx);
    const int64_t n = lbm::at(d, i, j);
    dst[k] = (double)src[n] + (base ? (double)base[n] : 0.0);
}

template <typename R>
int get_field_device(lbm_handle* h, int field, double* dst) {
    Offset off;
    R* p = field_ptr<R>(h, field, &off);
    if (!p || !dst) return LBM_EINVAL;
    const R* base = off == OFF_G ? h->st<R>().hb : nullptr;
    const int64_t n = (int64_t)h->dev.nx * h->dev.ny;
    k_field_out<R><<<(unsigned)((n + NT - 1) / NT), NT, 0, h->stream>>>(h->dev, p, base, dst);
    LAUNCHCHK(h);
    return LBM_OK;
}

template <typename R>
int get_set_field(lbm_handle* h, int field, double* buf, bool get) {
    Offset off;
    R* p = field_ptr<R>(h, field, &off);
    if (!p || !buf) return LBM_EINVAL;
    return copy_planes<R>(h, p, buf, 1, get, off);
}

template <typename R>
int get_set_pop(lbm_handle* h, int set, double* buf, bool get) {
    int nq = 0;
    Offset off;
    R* p = pop_ptr<R>(h, set, &nq, &off);
    if (!p || !buf) return LBM_EINVAL;
    return copy_planes<R>(h, p, buf, nq, get, off);
}

// FP16-storage form: the binary16 deviations of f, h or g decoded on the host with the bases
// the kernels use (the zero-velocity equilibria of the node's stored moments, evaluated in
// float by the same operations) and the exponent the current buffer was written with; the
// enthalpy base is added to the g rest link as for the FP32 form.  The D2Q5 links are FP32
// pairs, read as in that form.
float rest16(int set, int q, float a, float b, float cref) {
    const double w = q == 0 ? lbm::W0 : (q < 5 ? lbm::WA : lbm::WD);
    if (set == LBM_POP_F) return (float)w * a;
    if (set == LBM_POP_H) return ((float)(q == 0 ? w - 1.0 : w) * 3.0f) * a;
    return q == 0 ? (a - cref * b) + (float)lbm::W0 * (cref * b) : (float)w * (cref * b);
}

int get_pop16(lbm_handle* h, int set, double* host) {
    if (set == LBM_POP_L) return get_set_pop<float>(h, set, host, true);
    if (set < LBM_POP_F || set > LBM_POP_G || !host) return LBM_EINVAL;
    int rc = fetch_ctl(h);
    if (rc) return rc;
    const float inv = std::ldexp(1.f, -h->hctl->hexp[set][h->sp]);
    const Dev& d = h->dev;
    State<float>& s = h->sf;
    const int sp = h->sp;
    const size_t nx = (size_t)d.nx, pitch = (size_t)d.pitch, per = nx * (size_t)d.ny;
    const size_t plane = (size_t)d.plane;
    const float* sets[] = {s.f[sp], s.h[sp], s.g[sp]};
    std::vector<lbm::half_t> blk(9 * plane);
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(blk.data(), sets[set], blk.size() * sizeof(lbm::half_t), hipMemcpyDeviceToHost));
    const float* moment = set == LBM_POP_F ? s.psi[sp] : (set == LBM_POP_H ? s.p[sp] : s.H[sp]);
    std::vector<float> a, b, hb;
    rc = block_to_host<float>(h, a, moment, plane);
    if (!rc && set == LBM_POP_G) rc = block_to_host<float>(h, b, s.T[sp], plane);
    if (!rc && set == LBM_POP_G) rc = block_to_host<float>(h, hb, s.hb, plane);
    if (rc) return rc;
    const float cref = (float)d.Cref;
    for (int q = 0; q < 9; q++)
        for (size_t k = 0; k < per; k++) {
            const size_t n = (k / nx) * pitch + k % nx;
            const float base = rest16(set, q, a[n], set == LBM_POP_G ? b[n] : 0.f, cref);
            const float v = base + (float)blk[q * plane + n] * inv;
            host[q * per + k] = (double)v + (set == LBM_POP_G && q == 0 ? (double)hb[n] : 0.0);
        }
    return LBM_OK;
}

}  // namespace

// Streaming copy for lbm_time_copy: each thread moves four 16-byte words per pass, all loads
// issued before the stores.
__global__ void __launch_bounds__(256) k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * 256 * 4;
    for (size_t i = (size_t)blockIdx.x * 256 * 4 + threadIdx.x; i < n; i += stride) {
        uint4 v[4];
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (i + (size_t)k * 256 < n) v[k] = src[i + (size_t)k * 256];
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (i + (size_t)k * 256 < n) dst[i + (size_t)k * 256] = v[k];
    }
}

extern "C" {

int lbm_workspace_bytes(const lbm_params* p, size_t* bytes) {
    int rc = validate(p);
    if (rc) return rc;
    if (!bytes) return LBM_EINVAL;
    Dev d = make_dev(p);
    *bytes = carve_bytes(p, d);
    return LBM_OK;
}

int lbm_launch_shapes(const lbm_params* p, int* sweep_block, int* sweep_waves, int* stage_rows) {
    int rc = validate(p);
    if (rc) return rc;
    if (!sweep_block || !sweep_waves || !stage_rows) return LBM_EINVAL;
    *sweep_block = sweep_m(p);
    *sweep_waves = sweep_w(p);
    *stage_rows = make_dev(p).hseg;
    return LBM_OK;
}

int lbm_init(const lbm_params* p, void* workspace, size_t bytes, void* stream, lbm_handle** out) {
    int rc = validate(p);
    if (rc) return rc;
    if (!workspace || !out || ((uintptr_t)workspace % ALIGN) != 0) return LBM_EINVAL;
    Dev d = make_dev(p);
    size_t need = carve_bytes(p, d);
    if (bytes < need) return LBM_ESPACE;
    lbm_handle* h = new (std::nothrow) lbm_handle();
    if (!h) return LBM_EINVAL;
    h->prm = *p;
    h->dev = d;
    h->prec = p->precision;
    h->nb = d.gx * d.gy;
    h->stream = (hipStream_t)stream;
    h->ws = (char*)workspace;
    h->ws_bytes = bytes;
    h->swm = sweep_m(p);
    h->swv = sweep_w(p);
    if (h->prec != LBM_FP64) {
        carve<float>(d, h->ws, &h->sf, h->prec == LBM_FP32_FP16STORE);
        h->dctl = h->sf.ctl;
        h->partials = h->sf.partials;
    } else {
        carve<double>(d, h->ws, &h->sd);
        h->dctl = h->sd.ctl;
        h->partials = h->sd.partials;
    }
    if (hipHostMalloc((void**)&h->hword, 2 * sizeof(unsigned long long), hipHostMallocCoherent) != hipSuccess) {
        delete h;
        return LBM_EHIP;
    }
    h->hword[0] = h->hword[1] = 0;
    if (hipHostMalloc((void**)&h->hctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
        (void)hipHostFree(h->hword);
        delete h;
        return LBM_EHIP;
    }
    std::memset(h->hctl, 0, sizeof(Ctl));
    rc = h->prec == LBM_FP32_FP16STORE ? init_state<float, true>(h)
         : h->prec == LBM_FP32          ? init_state<float>(h)
                                        : init_state<double>(h);
    if (rc && rc != LBM_ENOCONV) {
        lbm_destroy(h);
        return rc;
    }
    *out = h;  // also after a capped initial solve: the state is valid
    return rc;
}

int lbm_step(lbm_handle* h, int n) {
    if (!h || h->spent) return LBM_ESTATE;
    if (n < 0) return LBM_EINVAL;
    for (int k = 0; k < n; k++) {
        int rc = h->prec == LBM_FP32_FP16STORE ? one_step<float, true>(h)
                 : h->prec == LBM_FP32          ? one_step<float>(h)
                                                : one_step<double>(h);
        if (rc) return rc;
    }
    return LBM_OK;
}

int lbm_solve_potential(lbm_handle* h, double tol, int max_sweeps, int* sweeps, double* resid) {
    if (!h || h->spent) return LBM_ESTATE;
    if (max_sweeps < 1) return LBM_EINVAL;
    return h->prec != LBM_FP64 ? solve_potential<float>(h, tol, max_sweeps, sweeps, resid)
                               : solve_potential<double>(h, tol, max_sweeps, sweeps, resid);
}

int lbm_diagnostics(lbm_handle* h, lbm_diag* out) {
    if (!h || h->spent) return LBM_ESTATE;
    if (!out) return LBM_EINVAL;
    int rc = h->prec == LBM_FP32_FP16STORE ? diagnostics<float, true>(h)
             : h->prec == LBM_FP32          ? diagnostics<float>(h)
                                            : diagnostics<double>(h);
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
    out->op_resid = c.op_res[0];
    out->op_resid_ramp = c.op_res[1];
    out->init_converged = h->init_conv;
    return c.nonfinite ? LBM_ENONFINITE : LBM_OK;
}

int lbm_get_field(lbm_handle* h, int field, double* dst) {
    if (!h || h->spent) return LBM_ESTATE;
    return h->prec != LBM_FP64 ? get_set_field<float>(h, field, dst, true)
                               : get_set_field<double>(h, field, dst, true);
}

int lbm_get_field_device(lbm_handle* h, int field, double* dst) {
    if (!h || h->spent) return LBM_ESTATE;
    return h->prec != LBM_FP64 ? get_field_device<float>(h, field, dst) : get_field_device<double>(h, field, dst);
}

int lbm_set_field(lbm_handle* h, int field, const double* src) {
    if (!h || h->spent) return LBM_ESTATE;
    double* s = const_cast<double*>(src);
    return h->prec != LBM_FP64 ? get_set_field<float>(h, field, s, false)
                               : get_set_field<double>(h, field, s, false);
}

int lbm_get_pop(lbm_handle* h, int set, double* dst) {
    if (!h || h->spent) return LBM_ESTATE;
    if (h->prec == LBM_FP32_FP16STORE) return get_pop16(h, set, dst);
    return h->prec == LBM_FP32 ? get_set_pop<float>(h, set, dst, true) : get_set_pop<double>(h, set, dst, true);
}

int lbm_set_pop(lbm_handle* h, int set, const double* src) {
    if (!h || h->spent) return LBM_ESTATE;
    double* s = const_cast<double*>(src);
    // FP16 storage: a write of f, h or g would have to be encoded against the running scales
    if (h->prec == LBM_FP32_FP16STORE && set != LBM_POP_L) return LBM_EINVAL;
    return h->prec != LBM_FP64 ? get_set_pop<float>(h, set, s, false) : get_set_pop<double>(h, set, s, false);
}

int lbm_sweep_log(lbm_handle* h, int* dst, int cap, int* count) {
    if (!h) return LBM_ESTATE;
    int n = (int)h->log.size();
    if (dst)
        for (int k = 0; k < n && k < cap; k++) dst[k] = h->log[k];
    if (count) *count = n;
    return LBM_OK;
}

// Checkpoint image: header, sweep log, then the used workspace bytes verbatim (every plane,
// partial sum and the control block are workspace-relative, so a handle of the same
// parameters can take the image).
namespace {
struct CkptHeader {
    uint64_t magic;
    int32_t version, nx, ny, precision, sweep_block, sweep_waves;
    int32_t sp, lcur, kprev, noconv, last_sweeps, nlog;
    int64_t step;
    double last_resid;
    uint64_t ws_bytes;
    uint64_t params_digest;  // of every lbm_params value: an image restores only into its own case
    int32_t init_conv, lbswap;
};
constexpr uint64_t CKPT_MAGIC = 0x4c424d434b505431ull;  // "LBMCKPT1"
constexpr int32_t CKPT_VERSION = 5;

// FNV-1a over the values of every lbm_params member (not its padding bytes).
uint64_t params_digest(const lbm_params& p) {
    uint64_t x = 0xcbf29ce484222325ull;
    auto mix8 = [&](uint64_t v) {
        for (int k = 0; k < 8; k++) {
            x ^= (v >> (8 * k)) & 0xff;
            x *= 0x100000001b3ull;
        }
    };
    auto i = [&](long long v) { mix8((uint64_t)v); };
    auto d = [&](double v) {
        uint64_t b;
        std::memcpy(&b, &v, sizeof b);
        mix8(b);
    };
    i(p.nx); i(p.ny); i(p.precision);
    d(p.W); d(p.M); d(p.gamma);
    d(p.rho_l); d(p.rho_g); d(p.rho_s); d(p.mu_l); d(p.mu_g); d(p.mu_s);
    d(p.cp_l); d(p.cp_g); d(p.cp_s); d(p.k_l); d(p.k_g); d(p.k_s); d(p.latent);
    d(p.T_w); d(p.T_g); d(p.eps_l); d(p.eps_g); d(p.eps_s); d(p.sig_l); d(p.sig_g); d(p.sig_s);
    d(p.phi_top); d(p.phi_bot); d(p.theta_deg);
    i(p.shape); d(p.R0); d(p.xc); d(p.yc); d(p.h0);
    d(p.poisson_tol); i(p.poisson_max_sweeps); i(p.readings);
    i(p.sweep_block); i(p.sweep_waves); i(p.stage_rows);
    return x;
}

size_t ckpt_bytes(const lbm_handle* h) {
    return sizeof(CkptHeader) + sizeof(int32_t) * h->log.size() + carve_bytes(&h->prm, h->dev);
}
}  // namespace

int lbm_checkpoint(lbm_handle* h, void* host, size_t* bytes) {
    if (!h || h->spent) return LBM_ESTATE;
    if (!bytes) return LBM_EINVAL;
    if (host) {
        int frc = flush_vl(h);  // the image carries the control block complete
        if (frc) return frc;
    }
    if (h->resid_stale) {
        int rc = fetch_ctl(h);
        if (rc) return rc;
    }
    size_t need = ckpt_bytes(h);
    if (!host) {
        *bytes = need;
        return LBM_OK;
    }
    if (*bytes < need) return LBM_ESPACE;
    CkptHeader hd{};
    hd.magic = CKPT_MAGIC;
    hd.version = CKPT_VERSION;
    hd.params_digest = params_digest(h->prm);
    hd.init_conv = h->init_conv;
    hd.lbswap = h->lbswap;
    hd.nx = h->dev.nx;
    hd.ny = h->dev.ny;
    hd.precision = h->prec;
    hd.sweep_block = h->swm;
    hd.sweep_waves = h->swv;
    hd.sp = h->sp;
    hd.lcur = h->lcur;
    hd.kprev = h->kprev;
    hd.noconv = h->noconv;
    hd.last_sweeps = h->last_sweeps;
    hd.nlog = (int32_t)h->log.size();
    hd.step = h->step;
    hd.last_resid = h->last_resid;
    hd.ws_bytes = carve_bytes(&h->prm, h->dev);
    char* out = (char*)host;
    std::memcpy(out, &hd, sizeof hd);
    out += sizeof hd;
    for (int v : h->log) {
        int32_t w = v;
        std::memcpy(out, &w, sizeof w);
        out += sizeof w;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(out, h->ws, hd.ws_bytes, hipMemcpyDeviceToHost));
    *bytes = need;
    return LBM_OK;
}

int lbm_restore(lbm_handle* h, const void* host, size_t bytes) {
    if (!h) return LBM_ESTATE;
    if (!host || bytes < sizeof(CkptHeader)) return LBM_EINVAL;
    CkptHeader hd;
    std::memcpy(&hd, host, sizeof hd);
    size_t ws = carve_bytes(&h->prm, h->dev);
    if (hd.magic != CKPT_MAGIC || hd.version != CKPT_VERSION || hd.nx != h->dev.nx || hd.ny != h->dev.ny ||
        hd.precision != h->prec || hd.sweep_block != h->swm || hd.sweep_waves != h->swv || hd.ws_bytes != ws ||
        hd.nlog < 0 || bytes < sizeof hd + sizeof(int32_t) * (size_t)hd.nlog + ws)
        return LBM_EINVAL;
    // buffer indices index the handle's plane tables: anything else is a corrupt image
    if (hd.sp < 0 || hd.sp > 1 || hd.lcur < 0 || hd.lcur > 2 || hd.kprev < 0 || hd.noconv < 0 || hd.step < 0 ||
        hd.lbswap < 0 || hd.lbswap > 1 ||
        hd.params_digest != params_digest(h->prm))
        return LBM_EINVAL;
    const char* in = (const char*)host + sizeof hd;
    std::vector<int> log(hd.nlog);
    for (int k = 0; k < hd.nlog; k++) {
        int32_t w;
        std::memcpy(&w, in, sizeof w);
        in += sizeof w;
        log[k] = w;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(h->ws, in, ws, hipMemcpyHostToDevice));
    h->sp = hd.sp;
    h->lcur = hd.lcur;
    h->kprev = hd.kprev;
    h->noconv = hd.noconv;
    h->last_sweeps = hd.last_sweeps;
    h->step = hd.step;
    h->last_resid = hd.last_resid;
    h->init_conv = hd.init_conv;
    if (hd.lbswap != h->lbswap) {  // the image's current base set is the handle's other one
        std::swap(h->sf.lb, h->sf.lbx);
        h->lbswap = hd.lbswap;
    }
    h->spent = false;
    h->resid_stale = false;
    h->vl_pending = false;
    h->log = std::move(log);
    return fetch_ctl(h);
}

int lbm_run_until_frozen(lbm_handle* h, int max_steps, int check_every, int* steps_done) {
    if (!h || h->spent) return LBM_ESTATE;
    if (max_steps < 0 || check_every < 1) return LBM_EINVAL;
    int k = 0;
    while (k < max_steps) {
        int rc = fetch_ctl(h);
        if (rc) return rc;
        if (h->hctl->t_fre > 0.0) break;
        int n = std::min(check_every, max_steps - k);
        rc = lbm_step(h, n);
        if (rc) return rc;
        k += n;
    }
    if (steps_done) *steps_done = k;
    return fetch_ctl(h);
}

int lbm_time_sweeps(lbm_handle* h, int n, float* ms) {
    if (!h) return LBM_ESTATE;
    if (n < 1 || !ms) return LBM_EINVAL;
    return h->prec != LBM_FP64 ? time_sweeps<float, 1>(h, n, ms) : time_sweeps<double, 1>(h, n, ms);
}

int lbm_time_stages(lbm_handle* h, int n, float* ms, int cap, int* nstages) {
    if (!h) return LBM_ESTATE;
    if (n < 1 || !nstages) return LBM_EINVAL;
    *nstages = NSTAGES;
    if (!ms) return LBM_OK;
    if (cap < NSTAGES) return LBM_EINVAL;
    h->spent = true;
    return h->prec == LBM_FP32_FP16STORE ? time_stages<float, true>(h, n, ms)
           : h->prec == LBM_FP32          ? time_stages<float>(h, n, ms)
                                          : time_stages<double>(h, n, ms);
}

const char* lbm_stage_name(int k) { return k >= 0 && k < NSTAGES ? STAGE_NAMES[k] : ""; }

int lbm_time_copy(void* dst, const void* src, size_t bytes, void* stream, int reps, float* ms) {
    if (!dst || !src || !ms || reps < 1 || bytes == 0 || bytes % 16 || (uintptr_t)dst % 16 ||
        (uintptr_t)src % 16)
        return LBM_EINVAL;
    const char *d0 = (const char*)dst, *s0 = (const char*)src;
    if (d0 < s0 + bytes && s0 < d0 + bytes) return LBM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const size_t n = bytes / 16;
    // enough workgroups for 8 per CU, each thread moving 4 x 16 B per pass
    const int blocks = (int)std::min<size_t>(2048, (n + 4 * 256 - 1) / (4 * 256));
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return LBM_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return LBM_EHIP;
    }
    k_copy16<<<blocks, 256, 0, st>>>((const uint4*)src, (uint4*)dst, n);  // warm-up
    hipError_t err = hipEventRecord(e0, st);
    for (int r = 0; r < reps && err == hipSuccess; r++) {
        k_copy16<<<blocks, 256, 0, st>>>((const uint4*)src, (uint4*)dst, n);
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e1, st);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float t = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return LBM_EHIP;
    *ms = t / (float)reps;
    return LBM_OK;
}

int lbm_destroy(lbm_handle* h) {
    if (!h) return LBM_OK;
    (void)hipStreamSynchronize(h->stream);
    if (h->hctl) (void)hipHostFree(h->hctl);
    if (h->hword) (void)hipHostFree(h->hword);
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

// ===========================================================================
// Autotuner of the potential-sweep shape.

namespace {

struct TuneKey {
    int nx, ny, prec;
    bool operator<(const TuneKey& o) const {
        return nx != o.nx ? nx < o.nx : ny != o.ny ? ny < o.ny : prec < o.prec;
    }
};
std::mutex tune_mu;
std::map<TuneKey, lbm_tune> tune_cache;

// Sweep shapes (sweeps per launch, waves per workgroup) worth timing.  Not 16 x 8: it is
// cheaper per sweep in back-to-back launches on small grids, which is what the tuner times,
// but a solve of a few sweeps loses with it (a coarser stopping launch, longer
// recomputations): 512 x 256 froze 14% slower with it.
constexpr int TUNE_MW[][2] = {{2, 4}, {2, 8}, {4, 4}, {4, 8}, {8, 4}, {8, 8}};
constexpr int TUNE_ROWS[] = {8, 16, 32, 64, 128};
// A candidate replaces the default shape only when the default is slower by more than this
// factor (the spread of repeated timings is about 1-2%): the choice then does not flip from
// run to run on near ties.
constexpr float TUNE_KEEP = 1.03f;

// Stage segment heights worth timing for this grid: the default first, then every candidate
// below the grid's height.
std::vector<int> tune_rows(const lbm_params* p) {
    lbm_params q = *p;
    q.stage_rows = 0;
    const Dev d0 = make_dev(&q);
    std::vector<int> rows{d0.hseg};
    for (int r : TUNE_ROWS)
        if (r != d0.hseg && r < p->ny) rows.push_back(r);
    if ((int)rows.size() > LBM_TUNE_MAXCAND) rows.resize(LBM_TUNE_MAXCAND);
    return rows;
}

// Workspace that holds any candidate's state (the largest over the shapes tried).
int tune_bytes(const lbm_params* p, size_t* need) {
    *need = 0;
    for (const auto& mw : TUNE_MW) {
        lbm_params q = *p;
        q.sweep_block = mw[0];
        q.sweep_waves = mw[1];
        size_t b = 0;
        int rc = lbm_workspace_bytes(&q, &b);
        if (rc) return rc;
        *need = std::max(*need, b);
    }
    for (int r : tune_rows(p)) {
        lbm_params q = *p;
        q.stage_rows = r;
        size_t b = 0;
        int rc = lbm_workspace_bytes(&q, &b);
        if (rc) return rc;
        *need = std::max(*need, b);
    }
    return LBM_OK;
}

int tune_shapes(const lbm_params* p, void* ws, size_t need, hipStream_t stream, int launches, lbm_tune* out) {
    lbm_tune r{};
    int rc = LBM_OK;
    float best = 0.f;
    for (const auto& mw : TUNE_MW) {
        const int m = mw[0], w = mw[1];
        lbm_params q = *p;
        q.sweep_block = m;
        q.sweep_waves = w;
        q.poisson_tol = -1.0;  // a short fixed initial solve: the timing needs no convergence
        q.poisson_max_sweeps = 2 * m;
        q.skip_initial_solve = 0;
        lbm_handle* h = nullptr;
        rc = lbm_init(&q, ws, need, stream, &h);
        if (rc) break;
        // launches tagged 2: a profile shows them apart from lbm_time_sweeps' (tag 1)
        float t0 = 0.f, t1 = 0.f;
        auto timed = [&](float* ms) {
            return h->prec != LBM_FP64 ? time_sweeps<float, 2>(h, launches * m, ms)
                                       : time_sweeps<double, 2>(h, launches * m, ms);
        };
        rc = timed(&t0);  // the first pass warms caches and code
        if (!rc) rc = timed(&t1);
        lbm_destroy(h);
        if (rc) break;
        float us = std::min(t0, t1) * 1e3f / (float)(launches * m);
        int k = r.ncand++;
        r.cand_block[k] = m;
        r.cand_waves[k] = w;
        r.us_per_sweep[k] = us;
        if (k == 0 || us < best) {
            best = us;
            r.sweep_block = m;
            r.sweep_waves = w;
        }
    }
    if (rc) return rc;
    // the default shape stays unless another is faster by more than timing noise
    for (int k = 0; k < r.ncand; k++)
        if (r.cand_block[k] == 8 && r.cand_waves[k] == 4 && r.us_per_sweep[k] <= TUNE_KEEP * best) {
            r.sweep_block = 8;
            r.sweep_waves = 4;
        }
    // stage segments, each timed as one f, flow and g stage (lbm_time_stages' launches)
    best = 0.f;
    for (int rows : tune_rows(p)) {
        lbm_params q = *p;
        q.stage_rows = rows;
        q.poisson_tol = -1.0;
        q.poisson_max_sweeps = 2;
        q.skip_initial_solve = 0;
        lbm_handle* h = nullptr;
        rc = lbm_init(&q, ws, need, stream, &h);
        if (rc) break;
        float ms[NSTAGES], total[2] = {0.f, 0.f};
        for (int pass = 0; pass < 2 && !rc; pass++) {
            rc = h->prec == LBM_FP32_FP16STORE ? time_stages<float, true>(h, launches, ms)
                 : h->prec == LBM_FP32          ? time_stages<float>(h, launches, ms)
                                                : time_stages<double>(h, launches, ms);
            for (int k = 0; k < NSTAGES; k++) total[pass] += ms[k];
        }
        lbm_destroy(h);
        if (rc) break;
        float us = std::min(total[0], total[1]) * 1e3f;
        int k = r.nrows++;
        r.cand_rows[k] = rows;
        r.us_per_step_stages[k] = us;
        if (k == 0 || us < best) {
            best = us;
            r.stage_rows = rows;
        }
    }
    if (rc) return rc;
    if (r.nrows > 0 && r.us_per_step_stages[0] <= TUNE_KEEP * best) r.stage_rows = r.cand_rows[0];  // the default
    *out = r;
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_autotune_workspace_bytes(const lbm_params* p, size_t* bytes) {
    int rc = validate(p);
    if (rc) return rc;
    if (!bytes) return LBM_EINVAL;
    return tune_bytes(p, bytes);
}

int lbm_autotune(const lbm_params* p, void* workspace, size_t bytes, void* stream, int launches, int flags,
                 lbm_tune* out) {
    int rc = validate(p);
    if (rc) return rc;
    if (!out || launches < 1) return LBM_EINVAL;
    TuneKey key{p->nx, p->ny, p->precision};
    if (!(flags & LBM_TUNE_FORCE)) {
        std::lock_guard<std::mutex> g(tune_mu);
        auto it = tune_cache.find(key);
        if (it != tune_cache.end()) {
            *out = it->second;
            out->cached = 1;
            return LBM_OK;
        }
    }
    size_t need = 0;
    rc = tune_bytes(p, &need);
    if (rc) return rc;
    if (!workspace || ((uintptr_t)workspace % ALIGN) != 0) return LBM_EINVAL;
    if (bytes < need) return LBM_ESPACE;
    lbm_tune r{};
    rc = tune_shapes(p, workspace, need, (hipStream_t)stream, launches, &r);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> g(tune_mu);
        tune_cache[key] = r;
    }
    *out = r;
    out->cached = 0;
    return LBM_OK;
}

}  // extern "C"

// ===========================================================================
// Batched form.

struct lbm_batch {
    int ncases = 0;
    int prec = LBM_FP64;
    int swm = 8;
    int swv = 4;
    hipStream_t stream = nullptr;
    std::vector<lbm_params> prm;
    std::vector<Dev> dev;
    std::vector<lbm::BatchCase<double>> cd;
    std::vector<lbm::BatchCase<float>> cf;
    void* table = nullptr;               // device BatchCase<R>[ncases]
    int* first_node = nullptr;           // device: first node-grid block of each case
    int* first_flow = nullptr;           // device: first flow-step window of each case
    int* first_fg = nullptr;             // device: first f/g-stage window of each case
    int* first_sw = nullptr;             // device: first sweep-grid block of each case
    int* lcur_d = nullptr;               // device: current potential buffer of each case
    int* lcur0_d = nullptr;              // device: buffer at the start of the running solve
    int* run_idx_d = nullptr;            // device: cases whose loops run (see batch_running)
    int* run_first_d = nullptr;          // device: their first sweep tiles in a launch
    double* tol_d = nullptr;
    int* maxsw_d = nullptr;
    lbm::SweepLaunch* fix_d = nullptr;
    Ctl* ctl_d = nullptr;                // ncases control blocks
    Ctl* ctl_h = nullptr;                // pinned mirror
    int node_blocks = 0, sweep_blocks = 0, flow_blocks = 0, fg_blocks = 0;
    std::vector<int> lcur, kprev;
    std::vector<int> run_idx_h, run_first_h;
    int run_blocks = 0;
    std::vector<std::vector<int>> log;
    std::vector<int> frozen_sp;          // buffer parity of a frozen case's final state (-1: running)
    std::vector<int> init_conv;          // each case's initial solve met the stopping rule
    std::vector<long long> case_step;    // steps each case has taken
    int sp = 0;
    long long step = 0;
    bool graphs = false;
    hipGraphExec_t gexec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [stage A/B][sp]
    hipGraph_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    std::string err;
};

namespace {

struct BatchLayout {
    std::vector<size_t> off;   // byte offset of each case's state
    size_t table, first_node, first_flow, first_fg, first_sw, lcur, lcur0, run_idx, run_first, tol, maxsw, fix, ctl,
        total;
};

int batch_validate(int ncases, const lbm_params* cases) {
    if (ncases < 1 || !cases) return LBM_EINVAL;
    for (int c = 0; c < ncases; c++) {
        int rc = validate(&cases[c]);
        if (rc) return rc;
        if (cases[c].precision != cases[0].precision || sweep_m(&cases[c]) != sweep_m(&cases[0]) ||
            sweep_w(&cases[c]) != sweep_w(&cases[0]) ||
            cases[c].skip_initial_solve != cases[0].skip_initial_solve)
            return LBM_EINVAL;
    }
    return LBM_OK;
}

BatchLayout batch_layout(int ncases, const lbm_params* cases) {
    BatchLayout L;
    size_t off = 0;
    const bool f32 = cases[0].precision != LBM_FP64, h16 = cases[0].precision == LBM_FP32_FP16STORE;
    for (int c = 0; c < ncases; c++) {
        L.off.push_back(off);
        Dev d = make_dev(&cases[c]);
        off = round_up(off + (f32 ? carve<float>(d, nullptr, nullptr, h16) : carve<double>(d, nullptr, nullptr)), ALIGN);
    }
    size_t cs = f32 ? sizeof(lbm::BatchCase<float>) : sizeof(lbm::BatchCase<double>);
    auto take = [&](size_t bytes) { size_t r = off; off = round_up(off + bytes, ALIGN); return r; };
    L.table = take(cs * ncases);
    L.first_node = take(sizeof(int) * ncases);
    L.first_flow = take(sizeof(int) * ncases);
    L.first_fg = take(sizeof(int) * ncases);
    L.first_sw = take(sizeof(int) * ncases);
    L.lcur = take(sizeof(int) * ncases);
    L.lcur0 = take(sizeof(int) * ncases);
    L.run_idx = take(sizeof(int) * ncases);
    L.run_first = take(sizeof(int) * ncases);
    L.tol = take(sizeof(double) * ncases);
    L.maxsw = take(sizeof(int) * ncases);
    L.fix = take(sizeof(lbm::SweepLaunch) * ncases);
    L.ctl = take(sizeof(Ctl) * ncases);
    L.total = off;
    return L;
}

#define BHIP(b, x)                                                       \
    do {                                                                 \
        hipError_t e_ = (x);                                             \
        if (e_ != hipSuccess) {                                          \
            (b)->err = std::string(#x) + ": " + hipGetErrorString(e_);   \
            return LBM_EHIP;                                             \
        }                                                                \
    } while (0)

template <typename R> std::vector<lbm::BatchCase<R>>& bcases(lbm_batch* b);
template <> std::vector<lbm::BatchCase<double>>& bcases<double>(lbm_batch* b) { return b->cd; }
template <> std::vector<lbm::BatchCase<float>>& bcases<float>(lbm_batch* b) { return b->cf; }

template <typename R>
const lbm::BatchCase<R>* btable(lbm_batch* b) { return (const lbm::BatchCase<R>*)b->table; }

// The loops still running (not done, not frozen) as the host last read the control blocks:
// their case indices and first sweep tiles go to the device, and the batch's sweep launches
// and tests cover only them (a batch whose other cases have converged launches no workgroups
// for those).  The host vectors stay untouched until the stream has drained.
template <typename R>
int batch_running(lbm_batch* b, bool fresh) {
    b->run_idx_h.clear();
    b->run_first_h.clear();
    int nb = 0;
    for (int c = 0; c < b->ncases; c++) {
        const bool running = b->frozen_sp[c] < 0 && (fresh || !b->ctl_h[c].done);
        if (!running) continue;
        b->run_idx_h.push_back(c);
        b->run_first_h.push_back(nb);
        nb += b->dev[c].tbx * b->dev[c].tby;
    }
    b->run_blocks = nb;
    const int nr = (int)b->run_idx_h.size();
    if (nr) {
        BHIP(b, hipMemcpyAsync(b->run_idx_d, b->run_idx_h.data(), sizeof(int) * nr, hipMemcpyHostToDevice, b->stream));
        BHIP(b, hipMemcpyAsync(b->run_first_d, b->run_first_h.data(), sizeof(int) * nr, hipMemcpyHostToDevice,
                               b->stream));
    }
    return LBM_OK;
}

template <typename R>
void batch_sweep(lbm_batch* b, int t) {
    const int nr = (int)b->run_idx_h.size();
    if (!nr) return;
    with_shape(b->swm, b->swv, [&](auto M, auto WV) {
        // one test block per running case, then the tiles of every running case
        lbm::kb_sweep<M, R, WV><<<b->run_blocks + nr, 64 * WV, 0, b->stream>>>(
            btable<R>(b), b->run_first_d, nr, b->lcur0_d, t, b->run_idx_d);
    });
}

template <typename R>
void batch_test(lbm_batch* b, int t) {
    auto tb = btable<R>(b);
    const int nr = (int)b->run_idx_h.size();
    if (!nr) return;
    with_shape(b->swm, 4, [&](auto M, auto) {
        lbm::kb_sweep_test<decltype(M)::value, R><<<nr, lbm::TEST_NT, 0, b->stream>>>(tb, b->lcur0_d, t,
                                                                                    b->run_idx_d);
    });
}

template <typename R>
void batch_fix(lbm_batch* b) {
    auto tb = btable<R>(b);
    with_shape(b->swm, b->swv, [&](auto M, auto WV) {
        lbm::kb_sweep_fix<M, R, WV><<<b->sweep_blocks, 64 * WV, 0, b->stream>>>(tb, b->first_sw, b->ncases, b->fix_d);
    });
}

// Lockstep potential loops of all cases.  Launch t performs sweeps t*M+1.. of every case
// that is still running (and, in one extra block per case, tests its launch t-1); a batch of
// launches ends with a one-block-per-case test of its last launch, then the host reads
// all control blocks.  Finished cases whose final sweep was not the last of its launch
// are recomputed together in one launch.
template <typename R>
int batch_sweeps(lbm_batch* b, int min_sweeps) {
    int nc = b->ncases;
    if (std::is_same<R, float>::value) {
        lbm::kb_rebase<R><<<b->node_blocks, NT, 0, b->stream>>>(btable<R>(b), b->first_node, nc, b->sp, b->lcur_d);
        lbm::kb_sweep_prep<R><<<b->node_blocks, NT, 0, b->stream>>>(btable<R>(b), b->first_node, nc, b->sp,
                                                                   b->lcur_d);
    }
    BHIP(b, hipMemcpyAsync(b->lcur0_d, b->lcur.data(), sizeof(int) * nc, hipMemcpyHostToDevice, b->stream));
    lbm::kb_ctl_reset<R><<<(nc + 63) / 64, 64, 0, b->stream>>>(btable<R>(b), nc, b->tol_d, min_sweeps, b->maxsw_d);
    BHIP(b, hipGetLastError());
    int rc = batch_running<R>(b, true);
    if (rc) return rc;
    int kmax = *std::max_element(b->kprev.begin(), b->kprev.end());
    int maxmax = 0;
    for (auto& p : b->prm) maxmax = std::max(maxmax, p.poisson_max_sweeps);
    int tmax = (maxmax + b->swm - 1) / b->swm;  // launches that reach every case's cap
    int nlaunch = kmax > 0 ? std::min(256, (kmax + b->swm - 1) / b->swm + 1) : 1;
    int grow = 1, t = 0;
    const bool rebasing = std::is_same<R, float>::value;
    const int reb = lbm::REBASE_SWEEPS / b->swm;  // launches between FP32 rebase points
    for (;;) {
        for (int c = 0; c < nlaunch && t < tmax; c++, t++) {
            if (rebasing && c > 0 && t % reb == 0) break;
            batch_sweep<R>(b, t);
        }
        batch_test<R>(b, t - 1);
        BHIP(b, hipGetLastError());
        BHIP(b, hipMemcpyAsync(b->ctl_h, b->ctl_d, sizeof(Ctl) * nc, hipMemcpyDeviceToHost, b->stream));
        BHIP(b, hipStreamSynchronize(b->stream));
        bool all = true;
        for (int c = 0; c < nc; c++) all = all && b->ctl_h[c].done;
        if (all) break;
        if (t >= tmax) {
            b->err = "potential loops ended without a decision";
            return LBM_EHIP;
        }
        rc = batch_running<R>(b, false);
        if (rc) return rc;
        if (rebasing && t % reb == 0) {
            lbm::kb_rebase_running<R><<<b->node_blocks, NT, 0, b->stream>>>(btable<R>(b), b->first_node, nc,
                                                                            b->lcur0_d, t);
            lbm::kb_sweep_prep<R><<<b->node_blocks, NT, 0, b->stream>>>(btable<R>(b), b->first_node, nc, b->sp,
                                                                       b->lcur_d);
        }
        nlaunch = grow;
        grow = std::min(grow * 2, 256);
    }
    std::vector<lbm::SweepLaunch> fix(nc);
    bool any = false;
    for (int c = 0; c < nc; c++) {
        if (b->frozen_sp[c] >= 0) {
            fix[c] = lbm::SweepLaunch{};
            continue;
        }
        const Ctl& ct = b->ctl_h[c];
        int f = ct.fix_launch;
        int src = (b->lcur[c] + f) % 3;
        int nsw_f = std::min(b->swm, b->prm[c].poisson_max_sweeps + 1 - (f * b->swm + 1));
        int final_buf = (src + 1) % 3;
        fix[c] = lbm::SweepLaunch{};
        if (ct.fix_n != nsw_f) {
            fix[c].src = src;
            fix[c].dst = (src + 2) % 3;
            fix[c].nsw = ct.fix_n;
            fix[c].k0 = f * b->swm + 1;
            fix[c].force = 1;
            final_buf = fix[c].dst;
            any = true;
        }
        b->lcur[c] = final_buf;
        b->kprev[c] = ct.count;
        b->log[c].push_back(ct.count);
    }
    if (any) {
        BHIP(b, hipMemcpyAsync(b->fix_d, fix.data(), sizeof(lbm::SweepLaunch) * nc, hipMemcpyHostToDevice, b->stream));
        batch_fix<R>(b);
        BHIP(b, hipGetLastError());
    }
    BHIP(b, hipMemcpyAsync(b->lcur_d, b->lcur.data(), sizeof(int) * nc, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

// The stages before (A) and after (B) the potential loop, for buffer parity sp (H: the f, h
// and g sets in binary16).
template <typename R, bool H = false>
void batch_stage(lbm_batch* b, int which, int sp) {
    auto tb = btable<R>(b);
    int nc = b->ncases;
    if (which == 0) {
        lbm::kb_f_fused<R, H><<<b->fg_blocks, NT, 0, b->stream>>>(tb, b->first_fg, nc, sp, b->lcur_d);
    } else {
        lbm::kb_h_fused<R, H><<<b->flow_blocks, NT, 0, b->stream>>>(tb, b->first_flow, nc, sp, b->lcur_d);
        lbm::kb_g_stream<R, H><<<b->fg_blocks, NT, 0, b->stream>>>(tb, b->first_fg, nc, sp, b->lcur_d);
        lbm::kb_vl_finalize<R><<<nc, NT, 0, b->stream>>>(tb, 0);
    }
}

template <typename R, bool H = false>
int batch_run_stage(lbm_batch* b, int which) {
    if (b->graphs) {
        BHIP(b, hipGraphLaunch(b->gexec[which][b->sp], b->stream));
    } else {
        batch_stage<R, H>(b, which, b->sp);
        BHIP(b, hipGetLastError());
    }
    return LBM_OK;
}

template <typename R, bool H = false>
int batch_capture(lbm_batch* b) {
    for (int which = 0; which < 2; which++)
        for (int sp = 0; sp < 2; sp++) {
            BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            batch_stage<R, H>(b, which, sp);
            BHIP(b, hipStreamEndCapture(b->stream, &b->graph[which][sp]));
            BHIP(b, hipGraphInstantiate(&b->gexec[which][sp], b->graph[which][sp], nullptr, nullptr, 0));
        }
    b->graphs = true;
    return LBM_OK;
}

template <typename R, bool H = false>
int batch_init_impl(lbm_batch* b, char* ws, const BatchLayout& L) {
    int nc = b->ncases;
    auto& cases = bcases<R>(b);
    cases.resize(nc);
    std::vector<int> fn(nc), fs(nc), ff(nc), fg(nc);
    std::vector<double> tol(nc);
    std::vector<int> maxsw(nc);
    Ctl* ctl = (Ctl*)(ws + L.ctl);
    for (int c = 0; c < nc; c++) {
        cases[c].d = b->dev[c];
        carve<R>(b->dev[c], ws + L.off[c], &cases[c].s, H);
        cases[c].s.ctl = ctl + c;
        fn[c] = b->node_blocks;
        fs[c] = b->sweep_blocks;
        ff[c] = b->flow_blocks;
        fg[c] = b->fg_blocks;
        b->fg_blocks += b->dev[c].gx * b->dev[c].hy;
        b->node_blocks += b->dev[c].gx * b->dev[c].gy;
        b->flow_blocks += b->dev[c].hx * b->dev[c].hy;
        b->sweep_blocks += b->dev[c].tbx * b->dev[c].tby;
        tol[c] = b->prm[c].poisson_tol;
        maxsw[c] = b->prm[c].poisson_max_sweeps;
    }
    BHIP(b, hipMemcpyAsync(b->table, cases.data(), sizeof(lbm::BatchCase<R>) * nc, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->first_node, fn.data(), sizeof(int) * nc, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->first_flow, ff.data(), sizeof(int) * nc, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->first_fg, fg.data(), sizeof(int) * nc, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->first_sw, fs.data(), sizeof(int) * nc, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->tol_d, tol.data(), sizeof(double) * nc, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->maxsw_d, maxsw.data(), sizeof(int) * nc, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->lcur_d, b->lcur.data(), sizeof(int) * nc, hipMemcpyHostToDevice, b->stream));
    for (int c = 0; c < nc; c++) k_ctl_zero<<<1, 1, 0, b->stream>>>(ctl + c);
    auto tb = btable<R>(b);
    lbm::kb_init<R, H><<<b->node_blocks, NT, 0, b->stream>>>(tb, b->first_node, nc, 0, b->lcur_d);
    lbm::kb_oml<R><<<b->node_blocks, NT, 0, b->stream>>>(tb, b->first_node, nc, 0, b->lcur_d);
    BHIP(b, hipGetLastError());
    b->init_conv.assign(nc, 1);
    if (b->prm[0].skip_initial_solve) {
        // the caller seeds and solves the potentials (lbm_batch_warm_start, lbm_batch_solve_potential)
        for (int c = 0; c < nc; c++) b->log[c].push_back(0);
    } else {
        int rc = batch_sweeps<R>(b, 2);
        if (rc) return rc;
        for (int c = 0; c < nc; c++) b->init_conv[c] = b->ctl_h[c].conv;
    }
    lbm::kb_vl0<R><<<b->fg_blocks, NT, 0, b->stream>>>(tb, b->first_fg, nc, 0, b->lcur_d);
    lbm::kb_vl_finalize<R><<<nc, NT, 0, b->stream>>>(tb, 1);
    BHIP(b, hipGetLastError());
    BHIP(b, hipStreamSynchronize(b->stream));
    if (b->stream) return batch_capture<R, H>(b);
    return LBM_OK;
}

template <typename R, bool H = false>
int batch_step_impl(lbm_batch* b) {
    int rc = batch_run_stage<R, H>(b, 0);
    if (rc) return rc;
    rc = batch_sweeps<R>(b, 1);
    if (rc) return rc;
    rc = batch_run_stage<R, H>(b, 1);
    if (rc) return rc;
    b->sp ^= 1;
    b->step++;
    for (int c = 0; c < b->ncases; c++)
        if (b->frozen_sp[c] < 0) b->case_step[c]++;
    return LBM_OK;
}

// Diagnostics and field reads reuse the single-case kernels on one case at a time.
// Potential solve of every case to its own rule, in lockstep launches (tau_l from the current
// psi and f_s first, as a step does after its f stage).
template <typename R>
int batch_solve(lbm_batch* b) {
    lbm::kb_oml<R><<<b->node_blocks, NT, 0, b->stream>>>(btable<R>(b), b->first_node, b->ncases, b->sp, b->lcur_d);
    BHIP(b, hipGetLastError());
    return batch_sweeps<R>(b, 1);
}

template <typename R>
int batch_case_handle(lbm_batch* b, int c, lbm_handle* h) {
    h->prm = b->prm[c];
    h->dev = b->dev[c];
    h->prec = b->prec;
    h->st<R>() = bcases<R>(b)[c].s;
    h->stream = b->stream;
    h->nb = b->dev[c].gx * b->dev[c].gy;
    h->sp = b->frozen_sp[c] >= 0 ? b->frozen_sp[c] : b->sp;
    h->lcur = b->lcur[c];
    h->swm = b->swm;
    h->swv = b->swv;
    h->dctl = bcases<R>(b)[c].s.ctl;
    h->partials = bcases<R>(b)[c].s.partials;
    h->step = b->case_step[c];
    h->hctl = b->ctl_h + c;
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_batch_workspace_bytes(int ncases, const lbm_params* cases, size_t* bytes) {
    int rc = batch_validate(ncases, cases);
    if (rc) return rc;
    if (!bytes) return LBM_EINVAL;
    *bytes = batch_layout(ncases, cases).total;
    return LBM_OK;
}

int lbm_batch_init(int ncases, const lbm_params* cases, void* workspace, size_t bytes, void* stream,
                   lbm_batch** out) {
    int rc = batch_validate(ncases, cases);
    if (rc) return rc;
    if (!workspace || !out || ((uintptr_t)workspace % ALIGN) != 0) return LBM_EINVAL;
    BatchLayout L = batch_layout(ncases, cases);
    if (bytes < L.total) return LBM_ESPACE;
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return LBM_EINVAL;
    char* ws = (char*)workspace;
    b->ncases = ncases;
    b->prec = cases[0].precision;
    b->swm = sweep_m(&cases[0]);
    b->swv = sweep_w(&cases[0]);
    b->stream = (hipStream_t)stream;
    b->prm.assign(cases, cases + ncases);
    for (int c = 0; c < ncases; c++) b->dev.push_back(make_dev(&cases[c]));
    b->table = ws + L.table;
    b->first_node = (int*)(ws + L.first_node);
    b->first_flow = (int*)(ws + L.first_flow);
    b->first_fg = (int*)(ws + L.first_fg);
    b->first_sw = (int*)(ws + L.first_sw);
    b->lcur_d = (int*)(ws + L.lcur);
    b->lcur0_d = (int*)(ws + L.lcur0);
    b->run_idx_d = (int*)(ws + L.run_idx);
    b->run_first_d = (int*)(ws + L.run_first);
    b->tol_d = (double*)(ws + L.tol);
    b->maxsw_d = (int*)(ws + L.maxsw);
    b->fix_d = (lbm::SweepLaunch*)(ws + L.fix);
    b->ctl_d = (Ctl*)(ws + L.ctl);
    b->lcur.assign(ncases, 0);
    b->kprev.assign(ncases, 0);
    b->log.assign(ncases, {});
    b->frozen_sp.assign(ncases, -1);
    b->case_step.assign(ncases, 0);
    if (hipHostMalloc((void**)&b->ctl_h, sizeof(Ctl) * ncases, hipHostMallocDefault) != hipSuccess) {
        delete b;
        return LBM_EHIP;
    }
    rc = b->prec == LBM_FP32_FP16STORE ? batch_init_impl<float, true>(b, ws, L)
         : b->prec == LBM_FP32          ? batch_init_impl<float>(b, ws, L)
                                        : batch_init_impl<double>(b, ws, L);
    if (rc) {
        lbm_batch_destroy(b);
        return rc;
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int n) {
    if (!b) return LBM_ESTATE;
    if (n < 0) return LBM_EINVAL;
    for (int k = 0; k < n; k++) {
        int rc = b->prec == LBM_FP32_FP16STORE ? batch_step_impl<float, true>(b)
                 : b->prec == LBM_FP32          ? batch_step_impl<float>(b)
                                                : batch_step_impl<double>(b);
        if (rc) return rc;
    }
    return LBM_OK;
}

int lbm_batch_run_until_frozen(lbm_batch* b, int max_steps, int* steps_done) {
    if (!b) return LBM_ESTATE;
    if (max_steps < 0) return LBM_EINVAL;
    int k = 0;
    for (; k < max_steps; k++) {
        bool all = true;
        for (int c = 0; c < b->ncases; c++) all = all && b->frozen_sp[c] >= 0;
        if (all) break;
        int rc = b->prec == LBM_FP32_FP16STORE ? batch_step_impl<float, true>(b)
                 : b->prec == LBM_FP32          ? batch_step_impl<float>(b)
                                                : batch_step_impl<double>(b);
        if (rc) return rc;
        // freezing detector of every case, after this step's liquid-volume update
        BHIP(b, hipMemcpyAsync(b->ctl_h, b->ctl_d, sizeof(Ctl) * b->ncases, hipMemcpyDeviceToHost, b->stream));
        BHIP(b, hipStreamSynchronize(b->stream));
        for (int c = 0; c < b->ncases; c++) {
            if (b->frozen_sp[c] >= 0 || !(b->ctl_h[c].t_fre > 0.0)) continue;
            b->frozen_sp[c] = b->sp;  // its final state is in the buffer just written
            const int one = 1;
            BHIP(b, hipMemcpyAsync(&b->ctl_d[c].frozen, &one, sizeof(int), hipMemcpyHostToDevice, b->stream));
            BHIP(b, hipStreamSynchronize(b->stream));
        }
    }
    if (steps_done) *steps_done = k;
    return LBM_OK;
}

int lbm_batch_diagnostics(lbm_batch* b, lbm_diag* per_case) {
    if (!b) return LBM_ESTATE;
    if (!per_case) return LBM_EINVAL;
    int worst = LBM_OK;
    for (int c = 0; c < b->ncases; c++) {
        lbm_handle h;
        if (b->prec != LBM_FP64) batch_case_handle<float>(b, c, &h); else batch_case_handle<double>(b, c, &h);
        h.log = b->log[c];
        h.last_sweeps = b->log[c].empty() ? 0 : b->log[c].back();
        h.last_resid = b->ctl_h[c].resid;
        h.init_conv = b->init_conv.empty() ? 1 : b->init_conv[c];
        int rc = lbm_diagnostics(&h, &per_case[c]);
        h.hctl = nullptr;  // owned by the batch
        if (rc == LBM_ENONFINITE) worst = rc;
        else if (rc) return rc;
    }
    return worst;
}

int lbm_batch_get_field(lbm_batch* b, int c, int field, double* dst) {
    if (!b) return LBM_ESTATE;
    if (c < 0 || c >= b->ncases) return LBM_EINVAL;
    lbm_handle h;
    if (b->prec != LBM_FP64) batch_case_handle<float>(b, c, &h); else batch_case_handle<double>(b, c, &h);
    int rc = lbm_get_field(&h, field, dst);
    h.hctl = nullptr;
    return rc;
}

int lbm_batch_sweep_log(lbm_batch* b, int c, int* dst, int cap, int* count) {
    if (!b) return LBM_ESTATE;
    if (c < 0 || c >= b->ncases) return LBM_EINVAL;
    int n = (int)b->log[c].size();
    if (dst)
        for (int k = 0; k < n && k < cap; k++) dst[k] = b->log[c][k];
    if (count) *count = n;
    return LBM_OK;
}

int lbm_batch_destroy(lbm_batch* b) {
    if (!b) return LBM_OK;
    (void)hipStreamSynchronize(b->stream);
    for (int w = 0; w < 2; w++)
        for (int s = 0; s < 2; s++) {
            if (b->gexec[w][s]) (void)hipGraphExecDestroy(b->gexec[w][s]);
            if (b->graph[w][s]) (void)hipGraphDestroy(b->graph[w][s]);
        }
    if (b->ctl_h) (void)hipHostFree(b->ctl_h);
    delete b;
    return LBM_OK;
}

}  // extern "C"

// ===========================================================================
// Learned warm start on a solver handle.

namespace {

bool coarse_ok(const lbm_handle* h, int f) {
    return f >= 1 && h->dev.nx % f == 0 && h->dev.ny % f == 0;
}

// The common divisor f of nx and ny that gives ny / f nearest `rows` coarse rows (ties: the
// larger f).
int coarse_factor(int nx, int ny, int rows) {
    int best = 1;
    double err = 1e300;
    for (int f = 1; f <= ny; f++) {
        if (nx % f || ny % f) continue;
        const double e = std::fabs((double)ny / f - rows);
        if (e <= err) {
            err = e;
            best = f;
        }
    }
    return best;
}

template <typename R>
int nn_features(lbm_handle* h, int f, float* x) {
    int nc = (h->dev.nx / f) * (h->dev.ny / f);
    lbm::k_nn_features<R><<<(nc + NT - 1) / NT, NT, 0, h->stream>>>(h->dev, h->st<R>(), h->sp, h->sp, f, x);
    LAUNCHCHK(h);
    return LBM_OK;
}

template <typename R>
int nn_target(lbm_handle* h, int f, float* t) {
    int nc = (h->dev.nx / f) * (h->dev.ny / f);
    lbm::k_nn_target<R><<<(nc + NT - 1) / NT, NT, 0, h->stream>>>(h->dev, h->st<R>(), h->lcur, f, t);
    LAUNCHCHK(h);
    return LBM_OK;
}

template <typename R>
int nn_seed(lbm_handle* h, int f, const float* y) {
    lbm::k_nn_seed<R><<<h->nb, NT, 0, h->stream>>>(h->dev, h->st<R>(), h->lcur, f, y);
    LAUNCHCHK(h);
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_nn_features(lbm_handle* h, int factor, float* x) {
    if (!h) return LBM_ESTATE;
    if (!x || !coarse_ok(h, factor)) return LBM_EINVAL;
    return h->prec != LBM_FP64 ? nn_features<float>(h, factor, x) : nn_features<double>(h, factor, x);
}

int lbm_nn_target(lbm_handle* h, int factor, float* t) {
    if (!h) return LBM_ESTATE;
    if (!t || !coarse_ok(h, factor)) return LBM_EINVAL;
    return h->prec != LBM_FP64 ? nn_target<float>(h, factor, t) : nn_target<double>(h, factor, t);
}

int lbm_nn_seed(lbm_handle* h, int factor, const float* y) {
    if (!h) return LBM_ESTATE;
    if (!y || !coarse_ok(h, factor)) return LBM_EINVAL;
    return h->prec != LBM_FP64 ? nn_seed<float>(h, factor, y) : nn_seed<double>(h, factor, y);
}

int lbm_warm_start(lbm_handle* h, lbm_nn* nnh, int factor) {
    if (!h || !nnh) return LBM_ESTATE;
    if (!coarse_ok(h, factor)) return LBM_EINVAL;
    int nxc = h->dev.nx / factor, nyc = h->dev.ny / factor;
    if ((int64_t)nxc * nyc > nnh->cap) return LBM_EINVAL;
    int rc = lbm_nn_features(h, factor, nnh->x);
    if (!rc) rc = nnapi::forward(nnh, nnh->x, nnh->y, 1, nyc, nxc, h->stream);
    if (rc) {
        if (rc == LBM_EHIP) h->err = nnh->err;
        return rc;
    }
    return lbm_nn_seed(h, factor, nnh->y);
}

int lbm_set_warm_start(lbm_handle* h, lbm_nn* nnh, int factor) {
    if (!h) return LBM_ESTATE;
    if (!nnh) {
        h->wnn = nullptr;
        h->wfactor = 0;
        return LBM_OK;
    }
    if (!coarse_ok(h, factor) || (int64_t)(h->dev.nx / factor) * (h->dev.ny / factor) > nnh->cap) return LBM_EINVAL;
    h->wnn = nnh;
    h->wfactor = factor;
    return LBM_OK;
}

int lbm_batch_nn_sample(lbm_batch* b, int c, int factor, float* x, float* t) {
    if (!b) return LBM_ESTATE;
    if (c < 0 || c >= b->ncases || !x || !t) return LBM_EINVAL;
    lbm_handle h;
    if (b->prec != LBM_FP64) batch_case_handle<float>(b, c, &h); else batch_case_handle<double>(b, c, &h);
    if (!coarse_ok(&h, factor)) return LBM_EINVAL;
    int rc = lbm_nn_features(&h, factor, x);
    if (!rc) rc = lbm_nn_target(&h, factor, t);
    if (!rc && hipStreamSynchronize(b->stream) != hipSuccess) rc = LBM_EHIP;
    if (rc) b->err = h.err;
    h.hctl = nullptr;
    return rc;
}

int lbm_batch_warm_start(lbm_batch* b, lbm_nn* nnh, int coarse_rows) {
    if (!b || !nnh) return LBM_ESTATE;
    if (coarse_rows < 1) return LBM_EINVAL;
    for (int c = 0; c < b->ncases; c++) {
        lbm_handle h;
        if (b->prec != LBM_FP64) batch_case_handle<float>(b, c, &h); else batch_case_handle<double>(b, c, &h);
        int rc = lbm_warm_start(&h, nnh, coarse_factor(h.dev.nx, h.dev.ny, coarse_rows));
        h.hctl = nullptr;
        if (rc) {
            b->err = h.err;
            return rc;
        }
    }
    return LBM_OK;
}

int lbm_batch_solve_potential(lbm_batch* b, int* max_sweeps_done) {
    if (!b) return LBM_ESTATE;
    int rc = b->prec != LBM_FP64 ? batch_solve<float>(b) : batch_solve<double>(b);
    if (rc) return rc;
    if (max_sweeps_done) {
        int k = 0;
        for (int c = 0; c < b->ncases; c++) k = std::max(k, b->log[c].empty() ? 0 : b->log[c].back());
        *max_sweeps_done = k;
    }
    return LBM_OK;
}

}  // extern "C"
