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
// Every kernel is a template on the real type R of storage and arithmetic: R = double
// (FP64 form) or R = float (FP32 form).  Reductions (potential residual, liquid volume,
// diagnostics) are FP64 in both.  In the FP32 form two population sets are stored as
// deviations from a per-node base, because their increments fall below an FP32 ulp of
// the raw values: the rest link of g and H minus h_b = psi rho_s L (the node's latent
// content, moved to the new psi every step; the rest link never streams, so this is
// exact), and each D2Q5 link as a pair (b_i, l_i) of an FP32 base and an FP32 remainder
// whose sum is the link.  The pair is renormalised (b_i <- b_i + l_i by an error-free
// two-sum) at the start of every potential solve and between batches of sweeps, so the
// sweeps work on remainders that hold only the change since then; the constant base terms
// of a launch are evaluated in FP64.  The FP64 form keeps no base: its arithmetic is the
// raw scheme.  The stages that move f, h and g also take a flag H: the FP32 form with those
// three sets stored in binary16 (see the FP16 storage section below).
//
// Blocks are 256 threads (4 waves of 64) covering a 64 x 4 tile.  The 1-D grid is
// remapped so that each of the 8 XCDs (which receive workgroups round-robin) works
// on one contiguous band of tiles: neighbouring tiles share that XCD's L2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

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
    int tbx, tby;                   // tiles of the blocked potential sweep in x and y
    int hx, hy, hseg;               // flow-step windows: strips in x, segments in y, rows each
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
    int done, count, conv;           // potential loop: finished, sweeps, converged
    int frozen;                      // batched runs to freezing: the case no longer advances
    int fix_launch, fix_n;           // launch holding the final sweep, and its sweeps up to it
    int fix_k0, fix_nsw;             // that launch's first sweep and its sweep count
    int min_sweeps, max_sweeps;
    double tol, resid;
    double V_l0, V_prev, t_fre;      // freezing-time detector
    long long step;
    int nonfinite;
    int final_buf;                   // potential buffer holding the last loop's final state
    double dsum[6];                  // sum psi, sum f, sum g, V_l, V_s, max |u|
    double front, height;
    double op_res[2];                // ||div(sigma grad phi)|| of phi and of the linear ramp
    // FP16 population storage: per set (f, h, g) and buffer, the scale exponent the buffer was
    // last written with and the largest |deviation| (FP32 bits) ever written into it
    int hexp[3][2];
    unsigned hmax[3][2];
};

// Arms the potential loop: clears its outcome and sets its stopping rule.
__device__ __forceinline__ void ctl_reset(Ctl* c, double tol, int min_sweeps, int max_sweeps) {
    c->fix_launch = 0;
    c->fix_n = 0;
    c->fix_k0 = 0;
    c->fix_nsw = 0;
    c->done = 0;
    c->count = 0;
    c->conv = 0;
    c->resid = 0.0;
    c->tol = tol;
    c->min_sweeps = min_sweeps;
    c->max_sweeps = max_sweeps;
}

// Offsets into the partial-sum array (nb = blocks of a node-parallel launch).
constexpr int SW_MAXM = 16;  // most sweeps one blocked launch performs
// FP32 potential base moves every REBASE_SWEEPS sweeps of a long solve (multiple of SW_MAXM)
constexpr int REBASE_SWEEPS = 256;
constexpr int DIAG_N = 9;  // per-tile diagnostics partials
__host__ __device__ constexpr int64_t part_vl(int nb) { return 0; }
__host__ __device__ constexpr int64_t part_diag(int nb) { return (int64_t)nb; }
__host__ __device__ constexpr int64_t part_sweep(int nb, int nbt, int slot) {
    return (int64_t)(1 + DIAG_N) * nb + (int64_t)slot * SW_MAXM * 2 * nbt;
}
__host__ __device__ constexpr int64_t part_total(int nb, int nbt) {
    return (int64_t)(1 + DIAG_N) * nb + (int64_t)2 * SW_MAXM * 2 * nbt;
}
constexpr int TEST_RANGES = 64;  // range sums of the convergence test (see k_sweep_test_part)
__host__ __device__ constexpr int64_t part_alloc(int nb, int nbt) {
    return part_total(nb, nbt) + (int64_t)2 * SW_MAXM * TEST_RANGES;
}

template <typename R>
__device__ __forceinline__ R clamp01(R x) { return x < R(0) ? R(0) : (x > R(1) ? R(1) : x); }

// Eq. (1) with psi clamped to [0, 1].
template <typename R>
__device__ __forceinline__ R mix(double s, double l, double g, R psi, R fs) {
    R pc = clamp01(psi);
    return fs * R(s) + (R(1) - fs) * pc * R(l) + (R(1) - fs) * (R(1) - pc) * R(g);
}

__device__ __forceinline__ int wrapx(int i, int nx) { return i < 0 ? i + nx : (i >= nx ? i - nx : i); }

__device__ __forceinline__ int64_t at(const Dev& d, int i, int j) { return (int64_t)j * d.pitch + i; }

// Field value with a ghost rule for rows -1 and ny (x already wrapped).
enum Ghost { GMIRROR = 0, GWET = 1, GPHI = 2 };
template <int G, typename R>
__device__ __forceinline__ R ghosted(const R* __restrict__ f, const Dev& d, int i, int j) {
    if (j < 0) {
        R b = f[i];
        if (G == GWET) return b + R(d.wet) * b * (R(1) - b);
        if (G == GPHI) return R(2.0 * d.phi_bot) - b;
        return b;
    }
    if (j >= d.ny) {
        R t = f[at(d, i, d.ny - 1)];
        if (G == GPHI) return R(2.0 * d.phi_top) - t;
        return t;  // mirror; psi meets the top wall at 90 degrees
    }
    return f[at(d, i, j)];
}

// 3x3 neighbourhood v[dy+1][dx+1] around (i, j).
template <int G, typename R>
__device__ __forceinline__ void load3(const R* __restrict__ f, const Dev& d, int i, int j, R v[3][3]) {
    int im = wrapx(i - 1, d.nx), ip = wrapx(i + 1, d.nx);
#pragma unroll
    for (int dy = -1; dy <= 1; dy++) {
        v[dy + 1][0] = ghosted<G, R>(f, d, im, j + dy);
        v[dy + 1][1] = ghosted<G, R>(f, d, i, j + dy);
        v[dy + 1][2] = ghosted<G, R>(f, d, ip, j + dy);
    }
}

// Eq. (36a) and (36b) on a 3x3 neighbourhood.  Differences from the centre are formed first:
// neighbouring values of a smooth field are close, so each difference is (nearly) exact and
// the rounding of the sums is relative to the differences, not to the field (an O(1) field
// such as psi or phi would otherwise carry an absolute rounding error of several ulps of 1
// into its Laplacian; in FP32 that is a relative error of 1e-5 to 1e-4 in the chemical
// potential and the free charge).
template <typename R>
__device__ __forceinline__ void grad_lap(const R v[3][3], R& gx, R& gy, R& lap) {
    const R wa = R(WA), wd = R(WD);
    const R c = v[1][1];
    const R e = v[1][2] - c, w = v[1][0] - c, n = v[2][1] - c, s = v[0][1] - c;
    const R ne = v[2][2] - c, nw = v[2][0] - c, sw = v[0][0] - c, se = v[0][2] - c;
    gx = R(3) * (wa * (e - w) + wd * ((ne - nw) + (se - sw)));
    gy = R(3) * (wa * (n - s) + wd * ((ne - se) + (nw - sw)));
    lap = R(6) * (wa * ((e + w) + (n + s)) + wd * ((ne + nw) + (sw + se)));
}

// The linear electrode ramp at row j (walls half a link outside the edge rows).
__device__ __forceinline__ double phi_lin(const Dev& d, int j) {
    return d.phi_bot + (d.phi_top - d.phi_bot) * (j + 0.5) / d.ny;
}

// XCD-aware block order: consecutive workgroup ids go to the 8 XCDs round-robin, so
// block b of a grid of nb blocks works on tile (b mod 8) * nb/8 + b/8, giving each XCD
// one contiguous band of tiles.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    int per = nb >> 3;
    return (per << 3) == nb ? (b & 7) * per + (b >> 3) : b;
}

// Node of this thread in tile `t` of the node grid.
__device__ __forceinline__ void node_of(const Dev& d, int t, int& i, int& j) {
    int bx = t % d.gx, by = t / d.gx;
    i = bx * TX + (threadIdx.x & (TX - 1));
    j = by * TY + (threadIdx.x / TX);
}

__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Neighbourhood staging for the streaming kernels: the collision inputs of a node tile
// (TX x TY) and of the one-node ring around it, gathered once into LDS so the nine pulls of a
// node read them there.  Slot (r, c) holds node (i0 - 1 + c, j0 - 1 + r) of the tile with
// origin (i0, j0), x wrapped (periodic); rows outside the grid stay unset (the pulls that
// would read them take the wall conditions instead).  Every thread of the block takes part.
constexpr int RX = TX + 2, RY = TY + 2, RN = RX * RY;
// tile with a two-node ring (stencils of the one-node ring's nodes)
constexpr int QX2 = TX + 4, QY2 = TY + 4, QN2 = QX2 * QY2;
template <typename T, typename F>
__device__ __forceinline__ void stage_ring(const Dev& d, int tile, T* ring, F&& load) {
    const int i0 = (tile % d.gx) * TX - 1, j0 = (tile / d.gx) * TY - 1;
    for (int k = threadIdx.x; k < RN; k += NT) {
        const int gj = j0 + k / RX;
        if (gj < 0 || gj >= d.ny) continue;
        int gi = (i0 + k % RX) % d.nx;
        if (gi < 0) gi += d.nx;
        ring[k] = load(at(d, gi, gj));
    }
    __syncthreads();
}
// Slot of this thread's node, and of its neighbour (i - cx, j - cy).
__device__ __forceinline__ int ring_self() { return (threadIdx.x / TX + 1) * RX + (threadIdx.x & (TX - 1)) + 1; }
__device__ __forceinline__ int ring_from(int self, int cx, int cy) { return self - cy * RX - cx; }

// Windows of the stage kernels.  A workgroup owns a strip of WX output columns and a segment
// of d.hseg rows and walks down it WR rows per pass, one wave per row, keeping what the
// stencils of the pass need in LDS rings of rows: fields WS = WX + 4 columns wide (the strip
// with a two-node halo), collision inputs WE = WX + 2 = 64 wide (one lane per column).  The
// grid columns of the window are tabulated once (x wrapped): window column c is grid column
// i0 - 3 + c.  Rows behind a pass are never evaluated again, so besides the x halo only a
// segment's first pass evaluates anything twice.
constexpr int WX = 62, WE = WX + 2, WS = WX + 4, WQ = WX + 6, WR = 4;
static_assert(WE == 64 && NT == 64 * WR, "one wave per window row");

// The f and g stages evaluate little per node and stream most of their bytes: their windows are
// strips of AX = 64 output columns aligned with the rows' cache lines, with collision inputs
// AE = AX + 2 and fields AS = AX + 4 columns wide (window column c is grid column i0 - 2 + c),
// d.gx strips by d.hy segments of d.hseg rows.
constexpr int AX = 64, AE = AX + 2, AS = AX + 4;
static_assert(WR * AS <= 2 * NT, "two staging items per thread at most");

// Column c (any integer) wrapped onto the periodic grid.
__device__ __forceinline__ int wrap_col(int c, int nx) {
    c %= nx;
    return c < 0 ? c + nx : c;
}
__device__ __forceinline__ int clamp_row(int y, int ny) { return y < 0 ? 0 : (y >= ny ? ny - 1 : y); }
// Ring slot of row y in a window whose segment starts at row jb (rows >= jb - 6).
__device__ __forceinline__ int slot6(int y, int jb) { return (y - jb + 6) % 6; }
// Blocks of the node-parallel per-block partial sums: enough for the node tiles and the windows.
__host__ __device__ inline int part_nb(const Dev& d) {
    const int a = d.gx * d.gy, b = d.hx * d.hy;
    return a > b ? a : b;
}

// v[dy+1][dx+1] = row_{dy}[c + dx], rows r0, r1, r2 = y - 1, y, y + 1.
template <typename T, typename U>
__device__ __forceinline__ void rows3(const T* r0, const T* r1, const T* r2, int c, U (&v)[3][3]) {
#pragma unroll
    for (int dx = -1; dx <= 1; dx++) {
        v[0][dx + 1] = r0[c + dx];
        v[1][dx + 1] = r1[c + dx];
        v[2][dx + 1] = r2[c + dx];
    }
}

// A field's value at row y in [-1, ny] from the value `raw` stored at row min(max(y, 0), ny - 1)
// of the same column: ghosted() split into its read and its ghost rule.
template <int G, typename R>
__device__ __forceinline__ R ghost_fix(R raw, const Dev& d, int y) {
    if (y < 0) {
        if (G == GWET) return raw + R(d.wet) * raw * (R(1) - raw);
        if (G == GPHI) return R(2.0 * d.phi_bot) - raw;
        return raw;
    }
    if (y >= d.ny) {
        if (G == GPHI) return R(2.0 * d.phi_top) - raw;
        return raw;
    }
    return raw;
}

// Wave-wide lane shifts by one lane on the VALU (DPP wave_shr / wave_shl): lane_up gives lane
// i the value of lane i - 1, lane_down the value of lane i + 1 (the lane at the end gets 0,
// written by the DPP bound control, so no register has to be cleared first).
__device__ __forceinline__ float lane_up(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_down(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_up(double x) {
    const long long v = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(v & 0xffffffffll), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0x138, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_down(double x) {
    const long long v = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(v & 0xffffffffll), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0x130, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
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
// N sums over a block of NTH threads in a fixed order: every thread parks its N values in
// sh[N][NTH]; G threads per value add fixed strided subsets, a butterfly over the G lanes
// combines them, and the N sums land in thread 0's v.  sh holds N * NTH + N doubles.  (Cheaper
// than N shuffle trees per wave: one LDS store per value and thread, one short butterfly.)
template <int N, int NTH>
__device__ __forceinline__ void block_sums_parked(double (&v)[N], double* sh) {
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < N; k++) sh[k * NTH + t] = v[k];
    __syncthreads();
    constexpr int G0 = NTH / N, G = G0 < 64 ? G0 : 64;
    static_assert((G & (G - 1)) == 0 && N * G <= NTH, "G lanes per value, within a wave");
    if (t < N * G) {
        const int k = t / G, p = t % G;
        double sum = 0.0;
        for (int q = p; q < NTH; q += G) sum += sh[k * NTH + q];
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
        if (p == 0) sh[N * NTH + k] = sum;
    }
    __syncthreads();
    if (t == 0)
#pragma unroll
        for (int k = 0; k < N; k++) v[k] = sh[N * NTH + k];
}
// The same sums for many values (N = 2M of a 16-sweep launch), in LDS of N doubles per wave:
// a butterfly over each wave, then thread 0 adds the waves in order.
template <int N, int NTH>
__device__ __forceinline__ void block_sums_waves(double (&v)[N], double* sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; k++) {
        double x = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) sh[w * N + k] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < N; k++) {
            double x = sh[k];
            for (int q = 1; q < NTH / 64; q++) x += sh[q * N + k];
            v[k] = x;
        }
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
template <typename R>
__device__ __forceinline__ R coll_f(int q, R fq, R psi, R ux, R uy, R Ax, R Ay, R md, const Dev& d) {
    R cu = R(QX[q]) * ux + R(QY[q]) * uy;
    R feq = R(QW[q]) * psi * (R(1) + R(3) * cu);
    R F = R(QW[q]) * (R(3) * (R(QX[q]) * Ax + R(QY[q]) * Ay) + psi * md);
    return fq - R(d.omf) * (fq - feq) + R(d.facf) * F;
}

// The same collision in deviation form (the FP32 forms, which store f_i - w_i psi): with
// f = w psi + dev at the source node, f - f_eq = dev - 3 w psi c.u, so the post-collision
// deviation from w psi is dev - omega (dev - 3 w psi c.u) + (1 - 1/(2 tau_f)) F: every rounding
// is relative to deviations, not to the O(w) populations.
template <typename R>
__device__ __forceinline__ R coll_f_dev(int q, R dq, R psi, R ux, R uy, R Ax, R Ay, R md, const Dev& d) {
    R cu = R(QX[q]) * ux + R(QY[q]) * uy;
    R neq = dq - R(QW[q]) * psi * (R(3) * cu);
    R F = R(QW[q]) * (R(3) * (R(QX[q]) * Ax + R(QY[q]) * Ay) + psi * md);
    return dq - R(d.omf) * neq + R(d.facf) * F;
}

template <typename R>
struct FIn {
    R psi, ux, uy, Ax, Ay, md;
};

// Flow, Eqs. (21)-(24).  (Ftx, Fty) = F~, (Gx, Gy) = F + rho f_solid.
template <typename R>
struct HIn {
    R p, rho, ux, uy, S, Ftx, Fty, Gx, Gy, om;
};
template <typename R>
__device__ __forceinline__ R coll_h(int q, R hq, const HIn<R>& a) {
    R cu = R(QX[q]) * a.ux + R(QY[q]) * a.uy;
    R uu = a.ux * a.ux + a.uy * a.uy;
    R s = R(QW[q]) * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu);
    R heq = R(q == 0 ? (QW[q] - 1.0) : QW[q]) * R(3) * a.p + a.rho * s;
    R cF = R(QX[q]) * a.Ftx + R(QY[q]) * a.Fty;
    R uF = a.ux * a.Ftx + a.uy * a.Fty;
    R cG = R(QX[q]) * a.Gx + R(QY[q]) * a.Gy;
    R Rq = R(QW[q]) * (a.S + R(3) * cG + R(9) * (cu * cF - R(CS2) * uF));
    return hq - a.om * (hq - heq) + (R(1) - R(0.5) * a.om) * Rq;
}

// Enthalpy, Eqs. (28)-(29) with the source weighted by omega_i.  H is the stored H - G.
template <typename R>
struct GIn {
    R H, T, C, ux, uy, om, Q;
};
template <typename R>
__device__ __forceinline__ R coll_g(int q, R gq, const GIn<R>& a, R Cref) {
    R uu = a.ux * a.ux + a.uy * a.uy;
    R geq;
    if (q == 0) {
        geq = a.H - Cref * a.T + R(W0) * (Cref * a.T - R(1.5) * a.C * a.T * uu);
    } else {
        R cu = R(QX[q]) * a.ux + R(QY[q]) * a.uy;
        geq = R(QW[q]) * (Cref * a.T + a.C * a.T * (R(3) * cu + R(4.5) * (cu * cu - R(CS2) * uu)));
    }
    return gq - a.om * (gq - geq) + (R(1) - R(0.5) * a.om) * R(QW[q]) * a.Q;
}

// Eq. (7) on the volumetric enthalpy, T_s = T_l = 0, latent heat psi * Lvol.  Hs is the
// stored enthalpy H - G with G the node's base (0 in FP64).
template <typename R>
__device__ __forceinline__ void invert(const Dev& d, R Hs, R G, R psi, R& T, R& fl) {
    // no fused multiply-add: Leff must be the rounded product the FP32 enthalpy base holds,
    // so that G - Leff cancels exactly when the base is current
#pragma clang fp contract(off)
    R pc = clamp01(psi);
    R Leff = pc * R(d.Lvol);
    if (Hs < -G) {
        fl = R(0);
        T = (Hs + G) / mix<R>(d.C_s, d.C_l, d.C_g, pc, pc);
    } else if (Hs <= Leff - G) {
        fl = Leff > R(0) ? (Hs + G) / Leff : R(1);
        T = R(0);
    } else {
        fl = R(1);
        T = (Hs + (G - Leff)) / mix<R>(d.C_s, d.C_l, d.C_g, pc, R(0));
    }
}

// ---------------------------------------------------------------------------
// FP16 population storage (FP32 arithmetic, template flag H of the stages that move f, h
// and g).  A population is stored as its deviation from the zero-velocity equilibrium of
// its node's stored moments (w_i psi for f, Eq. (18); the pressure part of Eq. (22) for h;
// Eq. (29) at u = 0 for g, with H the stored enthalpy) times a power-of-two scale of its
// set, rounded to binary16.  The stage that writes a set evaluates the base from the
// moments it stores beside it, and the stage that reads the set a step later from those
// stored moments, so the base cancels exactly and only the deviation is rounded.  The
// scale of a write puts the largest deviation ever written into the buffer it reads in
// [2^11, 2^12), sixteen times below the binary16 limit (binary16's relative precision does
// not depend on the scale; the scale only keeps values clear of overflow and of the
// subnormal range); a value beyond the limit saturates instead of overflowing.
using half_t = _Float16;
enum PopSet { PS_F = 0, PS_H = 1, PS_G = 2 };
constexpr int HS_TOP = 12, HS_EMIN = -16, HS_EMAX = 16;
constexpr float HALF_MAX = 65504.f;

// Scale exponent of a write whose set's previous maximum has the FP32 bits mbits (0: none).
__host__ __device__ constexpr int h16_exp(unsigned mbits) {
    if (mbits == 0) return HS_EMAX;
    const int e = (int)((mbits >> 23) & 0xff) - 127;  // maximum < 2^(e + 1)
    const int es = HS_TOP - 1 - e;
    return es < HS_EMIN ? HS_EMIN : (es > HS_EMAX ? HS_EMAX : es);
}
__device__ __forceinline__ float h16_get(const half_t* p, int64_t k, float base, float inv) {
    return base + (float)p[k] * inv;
}
__device__ __forceinline__ void h16_put(half_t* p, int64_t k, float dev, float sc) {
    float x = dev * sc;
    if (fabsf(x) > HALF_MAX) x = copysignf(HALF_MAX, x);  // NaN stays NaN
    p[k] = (half_t)x;
}
// Zero-velocity equilibria the deviations are taken from.
template <typename R>
__device__ __forceinline__ R f_rest(int q, R psi) { return R(QW[q]) * psi; }
template <typename R>
__device__ __forceinline__ R h_rest(int q, R p) { return R(q == 0 ? (QW[q] - 1.0) : QW[q]) * R(3) * p; }
template <typename R>
__device__ __forceinline__ R g_rest(int q, R H, R T, R Cref) {
#pragma clang fp contract(off)
    return q == 0 ? (H - Cref * T) + R(W0) * (Cref * T) : R(QW[q]) * (Cref * T);
}
// Folds the largest |deviation| of a block's write into *word, the running maximum (FP32
// bits) of every write into that buffer of the set.  Every thread of the block calls it, with
// 0 where it wrote nothing.  The word only grows, so a block whose maximum does not exceed a
// (possibly stale) cached read of it skips the atomic: after the first steps nearly every
// block does.
__device__ __forceinline__ void h16_note_max(unsigned* word, float m) {
    __shared__ float wm[NT / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float b = wm[0];
#pragma unroll
        for (int w = 1; w < NT / 64; w++) b = fmaxf(b, wm[w]);
        const unsigned u = __float_as_uint(b);
        if (u > *word) atomicMax(word, u);
    }
}
// Scales of one stage's read (buffer sp) and write (buffer sp ^ 1) of a set; thread 0 of the
// workgroup of the case's first tile (`first`) records the write's exponent (not block 0,
// which may serve another case or another task).  The write's exponent follows the running
// maximum of the writes into buffer sp, which no block of this launch changes (they fold into
// the other buffer's word), so every block derives the same exponent.
struct H16Scales {
    float inv, sc;
};
__device__ __forceinline__ H16Scales h16_scales(Ctl* c, int set, int sp, bool first) {
    const int eo = h16_exp(c->hmax[set][sp]);
    if (first && threadIdx.x == 0) c->hexp[set][sp ^ 1] = eo;
    return H16Scales{ldexpf(1.f, -c->hexp[set][sp]), ldexpf(1.f, eo)};
}

// ---------------------------------------------------------------------------
// Pointers of one stage.

template <typename R>
struct State {
    R* f[2];
    R* h[2];
    R* g[2];
    R* l[3];      // D2Q5 moving links E, N, W, S (the rest population never feeds phi)
    R* psi[2];
    R* ux[2];
    R* uy[2];
    R* p[2];
    R* H[2];
    R* T[2];
    R* fs[2];
    R* md[2];
    R* phi[3];         // raw phi
    R* lb;             // 4 base planes of the FP32 potential links (unused in FP64)
    R* lbx;            // FP32: the other base set (written by the solve-start renormalisation)
    R* dl;             // FP32: the 4 pulled base increments D of the current bases (see k_sweep_prep)
    R* pbp;            // FP32: the base potential phi_B = sum b / (1 - w_0)
    R* hb;             // enthalpy base of the FP32 rest link and H (unused in FP64)
    R* usx[2];
    R* usy[2];
    R *pux, *puy, *oml, *fl;
    double* partials;  // per-block FP64 reduction partials
    Ctl* ctl;
};

// ---------------------------------------------------------------------------
// Initialisation (Algorithm 1, first block): fields, equilibria in buffer 0.

template <typename R, bool H = false>
__device__ __forceinline__ void b_init(const Dev& d, const State<R>& s, int tile) {
#pragma clang fp contract(off)
    if (H && tile == 0 && threadIdx.x == 0)
        for (int k = 0; k < 3; k++) s.ctl->hexp[k][0] = HS_EMAX;  // the deviations written here are 0
    int i, j;
    node_of(d, tile, i, j);
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
    R psi = R(v);
    R pc = clamp01(psi);
    constexpr bool based = std::is_same<R, float>::value;
    R hb = based ? pc * R(d.Lvol) : R(0);
    R Hn = mix<R>(d.C_s, d.C_l, d.C_g, psi, R(0)) * R(d.T_g) + (pc * R(d.Lvol) - hb);
    if (based) s.hb[n] = hb;
    R T, fl;
    invert<R>(d, Hn, hb, psi, T, fl);
    R fs = pc * (R(1) - fl);
    double phi0 = d.phi_bot + (d.phi_top - d.phi_bot) * (j + 0.5) / d.ny;
    s.psi[0][n] = psi;
    s.ux[0][n] = 0; s.uy[0][n] = 0; s.usx[0][n] = 0; s.usy[0][n] = 0; s.p[0][n] = 0;
    s.H[0][n] = Hn; s.T[0][n] = T; s.fs[0][n] = fs; s.md[0][n] = 0; s.fl[n] = fl;
    s.pux[n] = 0; s.puy[n] = 0;
    R rho = mix<R>(d.rho_s, d.rho_l, d.rho_g, psi, fs);
    R C = mix<R>(d.C_s, d.C_l, d.C_g, psi, fs);
    HIn<R> hin{0, rho, 0, 0, 0, 0, 0, 0, 0, R(1)};
    GIn<R> gin{Hn, T, C, 0, 0, R(1), 0};
#pragma unroll
    for (int q = 0; q < 9; q++) {
        const R fq = R(QW[q]) * psi;
        const R hq = coll_h<R>(q, R(0), hin);  // omega = 1 returns h_eq
        const R gq = coll_g<R>(q, R(0), gin, R(d.Cref));
        if constexpr (H) {
            const float sc = ldexpf(1.f, HS_EMAX);
            h16_put((half_t*)s.f[0], q * d.plane + n, fq - f_rest<R>(q, psi), sc);
            h16_put((half_t*)s.h[0], q * d.plane + n, hq - h_rest<R>(q, R(0)), sc);
            h16_put((half_t*)s.g[0], q * d.plane + n, gq - g_rest<R>(q, Hn, T, R(d.Cref)), sc);
        } else {
            // FP32: f stored as its deviation from w_i psi (0 here)
            s.f[0][q * d.plane + n] = based ? fq - f_rest<R>(q, psi) : fq;
            s.h[0][q * d.plane + n] = hq;
            s.g[0][q * d.plane + n] = gq;
        }
    }
    double leq = LWA * phi0;
    R lbase = based ? R(leq) : R(0);
    R l = R(leq - (double)lbase);  // FP32: the remainder of the base (FP64: the link)
#pragma unroll
    for (int q = 0; q < 4; q++) {
        s.l[0][q * d.plane + n] = l;
        if (based) s.lb[q * d.plane + n] = lbase;
    }
    s.phi[0][n] = based ? R(phi0) : (l + l + l + l) * R(1.0 / (1.0 - LW0));
}
template <typename R, bool H = false>
__global__ void __launch_bounds__(NT) k_init(Dev d, State<R> s) {
    b_init<R, H>(d, s, xcd_tile(blockIdx.x, gridDim.x));
}

// The liquid volume of the state the g stage just wrote (its block partials, added in block
// order) and the freezing-time detector: mode 1 records V_l0 after initialisation; mode 0
// advances the step counter, and t_fre is the first step with V_l <= 1% of V_l0, interpolated
// linearly.  sh: NT / 64 doubles.
__device__ __forceinline__ void vl_finalize_body(const Dev& d, const double* partials, Ctl* c, int mode, double* sh) {
    const int nb = d.gx * d.hy;  // one partial per window of the g stage
    const double* pv = partials + part_vl(part_nb(d));
    double a = 0.0;
    for (int k = threadIdx.x; k < nb; k += NT) a += pv[k];
    a = block_sum(a, sh);
    if (threadIdx.x != 0) return;
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

// ---------------------------------------------------------------------------
// Stage 1a: A = d/dt(psi u) + c_s^2 lambda n at every node (Eqs. (19), (35)),
// then remember psi^n u^n for the next step.
// A at a node from psi^n around it (v), u^n and (psi u)^{n-1} there.  (psi u)^n itself is
// stored for the next step by the g stage (k_g_stream), after every reader of the old value.
// The coupling terms (gradients and Laplacians of Eq. (36), normals, the chemical potential,
// the forces and sources) are evaluated in FP64 from the stored fields in every form: on the
// gfx950 VALU an FP64 fused multiply-add issues at the rate of an unpacked FP32 one, so this
// costs the FP32 forms only conversions, while FP32 differences of O(1) fields at neighbouring
// nodes would inject errors far above one rounding of the stored values.  The FP32 forms keep
// FP32 arithmetic for the populations' collision, streaming and moments.
using K = double;
template <typename R>
__device__ __forceinline__ void to_k(const R (&v)[3][3], K (&w)[3][3]) {
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) w[a][b] = (K)v[a][b];
}

template <typename R>
__device__ __forceinline__ void a_term(const Dev& d, const R (&v)[3][3], R ux, R uy, R pux, R puy, R& Ax, R& Ay) {
    K w[3][3];
    to_k(v, w);
    K gx, gy, lap;
    grad_lap<K>(w, gx, gy, lap);
    K mag = sqrt(gx * gx + gy * gy);
    K nx = 0.0, ny = 0.0;
    if (mag > 1e-12) {
        nx = gx / mag;
        ny = gy / mag;
    }
    K ps = w[1][1];
    // psi clamped to [0, 1] in lambda as in Eq. (1): beyond [0, 1] the printed factor turns
    // negative and the counter term would steepen an overshoot (an instability) instead of
    // relaxing it
    const K pcl = clamp01(ps);
    K lam = 4.0 * pcl * (1.0 - pcl) / d.W;
    K px = ps * (K)ux, py = ps * (K)uy;
    Ax = R((px - (K)pux) + CS2 * lam * nx);
    Ay = R((py - (K)puy) + CS2 * lam * ny);
}

// Stage 1b: f pulled and collided at its source, half-way bounce-back at the walls;
// psi^{n+1} = sum f / (1 - mdot/2) (Eq. (20)); 1/tau_l for the sweeps.
// FP64 keeps the populations raw.  The FP32 forms (R = float; H: binary16 storage) keep each
// population as its deviation from w_i psi of its node and collide in deviation form: a link
// pulled from node y arrives as w_i psi(y) + e_i with e_i the collided deviation, psi^{n+1} is
// (sum_i w_i psi(y_i) + sum_i e_i) / (1 - mdot/2), and the stored deviation is
// w_i (psi(y_i) - psi^{n+1}) + e_i, a difference of neighbouring psi plus a small term.
// hv[q]: the stored value the pull of direction q reads (f_q at the source, or f_opp(q) at this
// node where the source is beyond a wall; FP16 storage: the binary16 value, not yet scaled);
// self, nbr(q): collision inputs of this node and of the source of direction q; mdn, fsn:
// this node's mdot and f_s.  H: returns the largest |deviation| written (0 otherwise).
template <typename R, bool H, typename NB>
__device__ __forceinline__ float f_stream_at(const Dev& d, const State<R>& s, int sp, int i, int j,
                                             const FIn<R>& self, NB&& nbr, const R (&hv)[9], H16Scales hs,
                                             R mdn, R fsn) {
    constexpr bool DEV = std::is_same<R, float>::value;
    const int64_t n = at(d, i, j);
    R* fdst = s.f[sp ^ 1];
    R sum = R(0), esum = R(0);
    R ev[DEV ? 9 : 1], pv[DEV ? 9 : 1];
#pragma unroll
    for (int q = 0; q < 9; q++) {
        int jj = j - QY[q];
        const bool wall = jj < 0 || jj >= d.ny;
        const int o = wall ? QOPP[q] : q;  // bounce-back: the node's own opposite link
        const FIn<R> a = wall ? self : nbr(q);
        R raw = hv[q];
        if constexpr (H) raw = 0.f + raw * hs.inv;
        if constexpr (DEV) {
            const R e = coll_f_dev<R>(o, raw, a.psi, a.ux, a.uy, a.Ax, a.Ay, a.md, d);
            ev[q] = e;
            pv[q] = a.psi;
            sum += f_rest<R>(q, a.psi);
            esum += e;
        } else {
            const R val = coll_f<R>(o, raw, a.psi, a.ux, a.uy, a.Ax, a.Ay, a.md, d);
            fdst[q * d.plane + n] = val;
            sum += val;
        }
    }
    R pn = (sum + esum) / (R(1) - R(0.5) * mdn);
    s.psi[sp ^ 1][n] = pn;
    R sig = mix<R>(d.sig_s, d.sig_l, d.sig_g, pn, fsn);
    s.oml[n] = R(1) / (sig / R(CS2) + R(0.5));
    float mx = 0.f;
    if constexpr (DEV) {
        // deviations from the equilibrium of the psi stored beside them
#pragma unroll
        for (int q = 0; q < 9; q++) {
            const R dv = R(QW[q]) * (pv[q] - pn) + ev[q];
            if constexpr (H) {
                mx = fmaxf(mx, fabsf(dv));
                h16_put((half_t*)fdst, q * d.plane + n, dv, hs.sc);
            } else {
                fdst[q * d.plane + n] = dv;
            }
        }
    }
    return mx;
}

// Stages 1a and 1b in one pass over a window (see AX): psi^n (wetting ghost) two rows ahead
// (AS columns), A and the other collision inputs of f one row ahead (AE columns), then the
// streaming of rows b .. b + 3.  The global reads of a pass's staging are issued during the
// previous pass's streaming, the pulls of f before the collision inputs are evaluated.
template <typename R>
struct FWin {
    R ps[6 * AS];      // psi^n, row y at slot slot6(y, jb)
    R in[6][6 * AE];   // collision inputs member by member (FIn order), rows as ps
    int col[AS];
};
template <typename R>
__device__ __forceinline__ FIn<R> fin_at(const FWin<R>& L, int o) {
    return FIn<R>{L.in[0][o], L.in[1][o], L.in[2][o], L.in[3][o], L.in[4][o], L.in[5][o]};
}
// Rows of pass t of an f or g window: fields rows [plo, phi), collision inputs rows [elo, ehi),
// streamed rows b .. b + 3 (t = -1: the rings' first rows only).
struct SPass {
    int b, plo, phi, elo, ehi;
};
__device__ __forceinline__ SPass s_pass(const Dev& d, int jb, int je, int t) {
    SPass a;
    a.b = jb + WR * t;
    a.plo = max(t < 0 ? jb - 2 : a.b + 2, -1);
    a.phi = min(min(a.b + 6, je + 2), d.ny + 1);
    a.elo = max(t < 0 ? jb - 1 : a.b + 1, 0);
    a.ehi = min(min(a.b + 5, je + 1), d.ny);
    return a;
}
template <typename R, bool H = false>
__device__ __forceinline__ void b_f_fused(const Dev& d, const State<R>& s, int sp, int tile) {
    __shared__ FWin<R> L;
    const int i0 = (tile % d.gx) * AX, jb = (tile / d.gx) * d.hseg;
    const int je = min(jb + d.hseg, d.ny);
    for (int c = threadIdx.x; c < AS; c += NT) L.col[c] = wrap_col(i0 - 2 + c, d.nx);
    H16Scales hs{};
    if constexpr (H) hs = h16_scales(s.ctl, PS_F, sp, tile == 0);
    float mx = 0.f;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const R* psi = s.psi[sp];
    const R* ux = s.ux[sp];
    const R* uy = s.uy[sp];
    const R* md = s.md[sp];
    const R* fsrc = s.f[sp];
    __syncthreads();  // L.col
    struct Fetch {
        R ps[2], ux[2], uy[2], pux[2], puy[2], md[2];
    } f;
    auto fetch = [&](int t) {
        const SPass a = s_pass(d, jb, je, t);
        const int np = (a.phi - a.plo) * AS, ne = (a.ehi - a.elo) * AE;
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int k = threadIdx.x + u * NT;
            if (k < np) f.ps[u] = psi[at(d, L.col[k % AS], clamp_row(a.plo + k / AS, d.ny))];
            if (k < ne) {
                const int64_t m = at(d, L.col[k % AE + 1], a.elo + k / AE);
                f.ux[u] = ux[m];
                f.uy[u] = uy[m];
                f.pux[u] = s.pux[m];
                f.puy[u] = s.puy[m];
                f.md[u] = md[m];
            }
        }
    };
    fetch(-1);
    for (int t = -1;; t++) {
        const SPass a = s_pass(d, jb, je, t);
        const int b = a.b;
        if (b >= je) break;
        const int np = (a.phi - a.plo) * AS, ne = (a.ehi - a.elo) * AE;
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int k = threadIdx.x + u * NT;
            if (k < np) {
                const int y = a.plo + k / AS;
                L.ps[slot6(y, jb) * AS + k % AS] = ghost_fix<GWET, R>(f.ps[u], d, y);
            }
        }
        __syncthreads();
        // this pass's streamed node (row b + wv, column i0 + lane): the nine values its pulls
        // read, its mdot and f_s
        const int j = b + wv, i = i0 + lane;
        const bool gv = t >= 0 && j < je && i < d.nx;
        R hv[9], mdn = R(0), fsn = R(0);
        if (gv) {
            const int64_t n = at(d, i, j);
#pragma unroll
            for (int q = 0; q < 9; q++) {
                const int jj = j - QY[q];
                const int64_t k = (jj < 0 || jj >= d.ny) ? QOPP[q] * d.plane + n
                                                         : q * d.plane + at(d, wrapx(i - QX[q], d.nx), jj);
                if constexpr (H) hv[q] = (R)((const half_t*)fsrc)[k];
                else hv[q] = fsrc[k];
            }
            mdn = md[n];
            fsn = s.fs[sp][n];
        }
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int k = threadIdx.x + u * NT;
            if (k >= ne) break;
            const int y = a.elo + k / AE, c = k % AE;
            R v[3][3];
            rows3(L.ps + slot6(y - 1, jb) * AS, L.ps + slot6(y, jb) * AS, L.ps + slot6(y + 1, jb) * AS, c + 1, v);
            R Ax, Ay;
            a_term<R>(d, v, f.ux[u], f.uy[u], f.pux[u], f.puy[u], Ax, Ay);
            const int o = slot6(y, jb) * AE + c;
            L.in[0][o] = v[1][1];
            L.in[1][o] = f.ux[u];
            L.in[2][o] = f.uy[u];
            L.in[3][o] = Ax;
            L.in[4][o] = Ay;
            L.in[5][o] = f.md[u];
        }
        __syncthreads();
        if (b + WR < je) fetch(t + 1);
        if (gv) {
            const int c = lane + 1;
            const int rm = slot6(j - 1, jb) * AE, r0 = slot6(j, jb) * AE, rp = slot6(j + 1, jb) * AE;
            auto nbr = [&](int q) -> FIn<R> {
                const int row = QY[q] > 0 ? rm : (QY[q] < 0 ? rp : r0);
                return fin_at(L, row + c - QX[q]);
            };
            mx = fmaxf(mx, f_stream_at<R, H>(d, s, sp, i, j, fin_at(L, r0 + c), nbr, hv, hs, mdn, fsn));
        }
    }
    if constexpr (H) h16_note_max(&s.ctl->hmax[PS_F][sp ^ 1], mx);
}
// fin = 1: one extra block, dispatched first so that it overlaps the others, finishes the
// previous step's liquid-volume sum and freezing-time detector meanwhile (a launch less per
// step; its fields of the control block are not the loop's).
template <typename R, bool H = false>
__global__ void __launch_bounds__(NT) k_f_fused_arm(Dev d, State<R> s, int sp, double tol, int min_sweeps,
                                                    int max_sweeps, int fin) {
    const int nb = gridDim.x - fin;
    if ((int)blockIdx.x < fin) {
        __shared__ double sh[NT / 64];
        vl_finalize_body(d, s.partials, s.ctl, 0, sh);
        return;
    }
    const int b = (int)blockIdx.x - fin;
    if (b == 0 && threadIdx.x == 0) ctl_reset(s.ctl, tol, min_sweeps, max_sweeps);
    b_f_fused<R, H>(d, s, sp, xcd_tile(b, nb));
}

// 1/tau_l = 1/(sigma/c_s^2 + 1/2) from the current psi and f_s (Sec. 3.4).
template <typename R>
__device__ __forceinline__ void b_oml(const Dev& d, const State<R>& s, int sp, int tile) {
    int i, j;
    node_of(d, tile, i, j);
    if (i >= d.nx || j >= d.ny) return;
    int64_t n = at(d, i, j);
    R sig = mix<R>(d.sig_s, d.sig_l, d.sig_g, s.psi[sp][n], s.fs[sp][n]);
    s.oml[n] = R(1) / (sig / R(CS2) + R(0.5));
}
template <typename R>
__global__ void __launch_bounds__(NT) k_oml(Dev d, State<R> s, int sp) {
    b_oml<R>(d, s, sp, xcd_tile(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// Blocked potential sweeps (Eqs. (31)-(34)).
//
// One launch advances the D2Q5 links by up to M sweeps.  A block of WV waves (4 or 8) owns
// a region of 64 columns x WV*SW_NPT rows; wave w holds rows [w*SW_NPT, (w+1)*SW_NPT) of the
// region, one column per lane, in registers.  Per sweep each node collides its four
// moving links towards w_i phi with its own 1/tau_l, then pulls: the E/W links come from
// the neighbouring lanes (wave-wide lane shifts), the N/S links from the rows above and
// below in the same lane, and only the rows at wave boundaries pass through LDS.  Walls:
// half-way anti-bounce-back at the electrodes; x is periodic (region columns wrap).
// After m sweeps the outer m columns/rows of the region are stale, so a block writes only
// its inner (64 - 2M) x (WV*SW_NPT - 2M) nodes.  For every sweep the block stores FP64 partial
// sums of |phi^k - phi^{k-1}|^2 and |phi^k|^2 over the nodes it writes; an extra block of
// the next launch adds them in block order and ends the loop at the first sweep that passes
// the test (that launch's sweeps up to it are then recomputed if it was not the last).
constexpr int SW_NPT = 8;
constexpr double INV_1MW0 = 1.0 / (1.0 - LW0);  // phi = (l_1 + l_2 + l_3 + l_4) / (1 - w_0), Eq. (34)

struct SweepLaunch {
    int src, dst;               // potential buffers (0..2)
    int nsw;                    // sweeps in this launch (0: only test the previous launch)
    int k0;                     // index of its first sweep within the solve (from 1)
    int slot;                   // partial-sum slot of this launch
    int prev_k0, prev_nsw, prev_slot;  // previous launch to test (prev_nsw = 0: none)
    int launch;                 // index of this launch within the solve
    int force;                  // run even if the loop has ended (recomputation)
    int devfix;                 // recompute the stopping launch up to the final sweep as the
                                // control block records it (src = the solve's first buffer);
                                // nothing if the loop has not ended or ended on a launch boundary
};

// Buffer of the stopping launch's input, and of the final state, for a loop that started
// from buffer lcur0 (launch t reads buffer (lcur0 + t) mod 3 and writes the next one; a
// recomputation writes the third).  The final sweep needs a recomputation unless it is the
// last of its launch.
__device__ __forceinline__ int stop_src(const Ctl* c, int lcur0) { return (lcur0 + c->fix_launch) % 3; }
__device__ __forceinline__ bool stop_recompute(const Ctl* c) { return c->fix_n != c->fix_nsw; }

// U: tiles fetched ahead (2 inside the sweep kernels, whose register budget it must fit; 4 in
// the one-workgroup test kernels).
template <int M, typename R, int NW = NT / 64, int U = 2>
__device__ __forceinline__ void sweep_sums(const Dev& d, const State<R>& s, const SweepLaunch& a, double* sh,
                                           int b0, int b1, double (&acc)[2 * M]) {
    int nbt = d.tbx * d.tby, nb = part_nb(d);
    const double* pv = s.partials + part_sweep(nb, nbt, a.prev_slot);
#pragma unroll
    for (int m = 0; m < 2 * M; m++) acc[m] = 0.0;
    // U tiles' partials are fetched before any is added (one memory latency per U tiles, not
    // per tile); the additions keep the order b, b + NTH, ..., so the sums are bitwise those
    // of one tile at a time
    constexpr int NTH = 64 * NW;
    int b = b0 + threadIdx.x;
    // one tile a pass for M > 8 (32 sums take as many registers as U = 2 at M = 8)
    constexpr int UU = M > 8 ? 1 : U;
    for (; b + (UU - 1) * NTH < b1; b += UU * NTH) {
        double v[UU][2 * M];
#pragma unroll
        for (int u = 0; u < UU; u++)
#pragma unroll
            for (int m = 0; m < M; m++) {
                const double* q = pv + ((int64_t)m * nbt + b + u * NTH) * 2;
                v[u][2 * m] = m < a.prev_nsw ? q[0] : 0.0;
                v[u][2 * m + 1] = m < a.prev_nsw ? q[1] : 0.0;
            }
#pragma unroll
        for (int u = 0; u < UU; u++)
#pragma unroll
            for (int m = 0; m < M; m++)
                if (m < a.prev_nsw) {
                    acc[2 * m] += v[u][2 * m];
                    acc[2 * m + 1] += v[u][2 * m + 1];
                }
    }
    for (; b < b1; b += NTH)
#pragma unroll
        for (int m = 0; m < M; m++)
            if (m < a.prev_nsw) {
                acc[2 * m] += pv[((int64_t)m * nbt + b) * 2];
                acc[2 * m + 1] += pv[((int64_t)m * nbt + b) * 2 + 1];
            }
    if constexpr (M > 8) block_sums_waves<2 * M, NTH>(acc, sh);
    else block_sums_parked<2 * M, NTH>(acc, sh);
}
// The stopping rule on the summed residuals of the tested launch (thread 0 only).
template <int M>
__device__ __forceinline__ void sweep_decide(Ctl* c, const SweepLaunch& a, const double (&acc)[2 * M]) {
    // a loop without early exits, unrolled: acc stays in registers (a run-time index would put
    // it in scratch memory); the sweeps after the stopping one are skipped
    const double tol = c->tol;
    const int min_sweeps = c->min_sweeps, max_sweeps = c->max_sweeps;
    double resid = 0.0;
    int count = 0, seen = 0, stop = 0, conv = 0, fix_n = 0;
#pragma unroll
    for (int m = 0; m < M; m++) {
        if (stop || m >= a.prev_nsw) continue;
        const double da = acc[2 * m], pa = acc[2 * m + 1];
        const double r = da == 0.0 ? 0.0 : (pa > 0.0 ? sqrt(da) / sqrt(pa) : INFINITY);
        const int j = a.prev_k0 + m;
        resid = r;
        count = j;
        seen = 1;
        conv = tol >= 0.0 && j >= min_sweeps && r <= tol;
        if (conv || j >= max_sweeps) {
            stop = 1;
            fix_n = m + 1;
        }
    }
    if (!seen) return;
    c->resid = resid;
    c->count = count;
    if (stop) {
        c->conv = conv;
        c->done = 1;
        c->fix_launch = a.launch - 1;
        c->fix_n = fix_n;
        c->fix_k0 = a.prev_k0;
        c->fix_nsw = a.prev_nsw;
    }
}
template <int M, typename R, int NW = NT / 64, int U = 2>
__device__ __forceinline__ void sweep_test(const Dev& d, const State<R>& s, const SweepLaunch& a, double* sh) {
    double acc[2 * M];
    sweep_sums<M, R, NW, U>(d, s, a, sh, 0, d.tbx * d.tby, acc);
    if (threadIdx.x == 0) sweep_decide<M>(s.ctl, a, acc);
}

// The test of the previous launch (a.prev_*) is not made here: the launches carry extra
// blocks for it (k_sweep_tb, kb_sweep).
// Shared doubles a sweep workgroup (or the test block beside it) uses for its sums.
template <int M, int WV>
constexpr int SWEEP_SHM = M > 8 ? 2 * 8 * 64 * WV : 2 * M * 64 * WV + 2 * M;
// Sweeps whose residual sums a sweep workgroup parks at once: a launch of more sweeps sums
// and empties the parking after every eighth (LDS for all 16 would halve the occupancy).
template <int M>
constexpr int SW_PARK = M > 8 ? 8 : M;

template <int M, typename R, int WV>
__device__ __forceinline__ void b_sweep_tb(const Dev& d, const State<R>& s, const SweepLaunch& ain, int tile,
                                           double* accs) {
    // no implicit contraction: the fused operations are written out, so the result does not
    // depend on how the compiler unrolls the M sweeps (bitwise equal for every launch shape)
#pragma clang fp contract(off)
    __shared__ R bup[2][WV][64], bdn[2][WV][64];
    // accs: each thread's FP64 residual sums of every sweep, parked at the end of the sweep
    // instead of in registers (16 accumulators would cost the kernel a wave per SIMD)
    constexpr int NTH = 64 * WV, PK = SW_PARK<M>;
    const Ctl* c = s.ctl;
    SweepLaunch a = ain;
    if (a.devfix) {
        if (!c->done || !stop_recompute(c)) return;
        a.src = stop_src(c, ain.src);
        a.dst = (a.src + 2) % 3;
        a.k0 = c->fix_k0;
        a.nsw = c->fix_n;
        a.force = 1;
        a.prev_nsw = 0;
    }
    if (c->done && !a.force) return;
    if (a.nsw > 0) {
        constexpr int OX = 64 - 2 * M, OY = WV * SW_NPT - 2 * M;
        const R inv = R(INV_1MW0), lw = R(LWA);
        int nbt = d.tbx * d.tby;
        int bx = tile % d.tbx, by = tile / d.tbx;
        // w (the wave) and everything derived from it is wave-uniform: scalar registers
        int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        int x0 = bx * OX - M, y0 = by * OY - M + w * SW_NPT;
        int graw = x0 + lane;
        int gi = graw % d.nx;
        if (gi < 0) gi += d.nx;
        const bool ownx = lane >= M && lane < M + OX && graw < d.nx;
        const R* ls = s.l[a.src];
        const int64_t P = d.plane;
        constexpr bool based = std::is_same<R, float>::value;
        // OMC = 1 - omega: the collision l - omega (l - w phi) is evaluated as
        // (1 - omega) l + omega w phi, the second term once per node
        R L1[SW_NPT], L2[SW_NPT], L3[SW_NPT], L4[SW_NPT], OMC[SW_NPT], PB[SW_NPT], PH[SW_NPT];
        // a launch of nsw < M sweeps needs only the rows within nsw of the written ones: the
        // others stay zero (never read from memory), which changes no written node
        auto needed = [&](int k) {
            const int r = w * SW_NPT + k, gj = y0 + k;
            return gj >= 0 && gj < d.ny && r >= M - a.nsw && r < M + OY + a.nsw;
        };
#pragma unroll
        for (int k = 0; k < SW_NPT; k++) {
            int gj = y0 + k;
            if (needed(k)) {
                int64_t n = at(d, gi, gj);
                L1[k] = ls[n];
                L2[k] = ls[P + n];
                L3[k] = ls[2 * P + n];
                L4[k] = ls[3 * P + n];
                OMC[k] = R(1) - s.oml[n];
            } else {
                L1[k] = L2[k] = L3[k] = L4[k] = OMC[k] = R(0);
            }
            PB[k] = R(0);
            PH[k] = (L1[k] + L2[k] + L3[k] + L4[k]) * inv;
        }
        // FP32 pair storage (link = b + l): the sweep works on the remainders l; the pulled
        // base increments D and phi_B are launch constants prepared by k_sweep_prep
        R D1[SW_NPT], D2[SW_NPT], D3[SW_NPT], D4[SW_NPT];
        if constexpr (based) {
#pragma unroll
            for (int k = 0; k < SW_NPT; k++) {
                int gj = y0 + k;
                if (needed(k)) {
                    int64_t n = at(d, gi, gj);
                    D1[k] = s.dl[n];
                    D2[k] = s.dl[P + n];
                    D3[k] = s.dl[2 * P + n];
                    D4[k] = s.dl[3 * P + n];
                    PB[k] = s.pbp[n];
                } else {
                    D1[k] = D2[k] = D3[k] = D4[k] = R(0);
                }
            }
        }
        const R wbot0 = R(2.0 * LWA * d.phi_bot), wtop0 = R(2.0 * LWA * d.phi_top);
        // block sums of the parked values of sweeps m0 .. m0 + PK - 1: G threads per value, each
        // adding a fixed strided subset, then a butterfly over the G lanes (a fixed order:
        // reproducible)
        double* pw = s.partials + part_sweep(part_nb(d), nbt, a.slot);
        auto park_sums = [&](int m0) {
            constexpr int G0 = NTH / (2 * PK), G = G0 < 64 ? G0 : 64;
            __syncthreads();
            const int t = threadIdx.x;
            if (t < 2 * PK * G) {
                const int v = t / G, p = t % G, m = m0 + v / 2;
                double sum = 0.0;
                for (int q = p; q < NTH; q += G) sum += accs[v * NTH + q];
#pragma unroll
                for (int off = G / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
                if (p == 0 && m < a.nsw) pw[((int64_t)m * nbt + tile) * 2 + (v & 1)] = sum;
            }
        };
        double rw[SW_NPT];  // 1: the row is written by this block (inner rows inside the domain)
#pragma unroll
        for (int k = 0; k < SW_NPT; k++) {
            const int r = w * SW_NPT + k, gj = y0 + k;
            rw[k] = (r >= M && r < M + OY && gj >= 0 && gj < d.ny) ? 1.0 : 0.0;
        }
        // M > 8: chunks of PK sweeps, each unrolled as a launch of PK sweeps
#pragma unroll 1
        for (int c0 = 0; c0 < M; c0 += PK) {
#pragma unroll
            for (int mm = 0; mm < PK; mm++) {
                const int m = c0 + mm;
                if (m >= a.nsw) break;
                R A1[SW_NPT], A2[SW_NPT], A3[SW_NPT], A4[SW_NPT];
                double accd = 0.0, accp = 0.0;
#pragma unroll
                for (int k = 0; k < SW_NPT; k++) {
                    // PH: phi of the current links (from the load, then from the previous sweep)
                    R e = lw * PH[k];
                    R q = fma_r(-OMC[k], e, e);  // omega w phi
                    // explicit fused multiply-adds, so every launch shape rounds them the same way
                    A1[k] = fma_r(OMC[k], L1[k], q);
                    A2[k] = fma_r(OMC[k], L2[k], q);
                    A3[k] = fma_r(OMC[k], L3[k], q);
                    A4[k] = fma_r(OMC[k], L4[k], q);
                }
                int par = mm & 1;  // = m & 1: c0 is a multiple of PK, which is even or M
                bup[par][w][lane] = A2[SW_NPT - 1];
                bdn[par][w][lane] = A4[0];
                __syncthreads();
                R below = w > 0 ? bup[par][w - 1][lane] : R(0);
                R above = w < WV - 1 ? bdn[par][w + 1][lane] : R(0);
#pragma unroll
                for (int k = 0; k < SW_NPT; k++) {
                    int gj = y0 + k;
                    R n1 = lane_up(A1[k]);
                    R n3 = lane_down(A3[k]);
                    R n2 = k > 0 ? A2[k - 1] : below;
                    R n4 = k < SW_NPT - 1 ? A4[k + 1] : above;
                    if constexpr (based) {
                        n1 = n1 + D1[k];
                        n3 = n3 + D3[k];
                        n2 = gj == 0 ? D2[k] - A4[k] : n2 + D2[k];
                        n4 = gj == d.ny - 1 ? D4[k] - A2[k] : n4 + D4[k];
                    } else {
                        if (gj == 0) n2 = wbot0 - A4[k];
                        if (gj == d.ny - 1) n4 = wtop0 - A2[k];
                    }
                    L1[k] = n1;
                    L2[k] = n2;
                    L3[k] = n3;
                    L4[k] = n4;
                    const R ph = (n1 + n2 + n3 + n4) * inv;
                    // rows count with the wave-uniform weight rw[k] (1 or 0: a scalar operand, no
                    // per-node select); the column mask ownx is applied when the sums are parked
                    double dd = (double)(ph - PH[k]);
                    double pr = based ? (double)ph + (double)PB[k] : (double)ph;
                    accd = __builtin_fma(dd * rw[k], dd, accd);
                    accp = __builtin_fma(pr * rw[k], pr, accp);
                    PH[k] = ph;
                }
                accs[(2 * mm) * NTH + threadIdx.x] = ownx ? accd : 0.0;
                accs[(2 * mm + 1) * NTH + threadIdx.x] = ownx ? accp : 0.0;
                // the parking is full and more sweeps follow: sum it (the next sweep's barrier
                // orders these reads before its stores)
                if constexpr (M > PK)
                    if (mm == PK - 1 && m + 1 < a.nsw) park_sums(c0);
            }
        }
        R* ld = s.l[a.dst];
        R* pd = s.phi[a.dst];
#pragma unroll
        for (int k = 0; k < SW_NPT; k++) {
            int gj = y0 + k;
            int r = w * SW_NPT + k;
            if (ownx && r >= M && r < M + OY && gj >= 0 && gj < d.ny) {
                int64_t n = at(d, gi, gj);
                ld[n] = L1[k];
                ld[P + n] = L2[k];
                ld[2 * P + n] = L3[k];
                ld[3 * P + n] = L4[k];
                pd[n] = based ? PB[k] + PH[k] : PH[k];
            }
        }
        park_sums(((a.nsw - 1) / PK) * PK);
    }
}

// One launch of the single-case loop: block 0 tests the previous launch (its partial sums are
// complete when the launch starts) and blocks 1 .. nb sweep their tiles meanwhile, which takes
// the test off the launch's critical path (20.2 us against 25.4 us per 8-sweep FP64 launch at
// 1024 x 512).  Blocks are dispatched in order, so the test starts first: the blocks that
// start after it has ended the loop exit at once, as the whole launch would have (their
// output is never used: the final state is the previous launch's, or recomputed from its
// input).
// Tag only separates launches in a profile (1: the timing entry point, 2: the autotuner),
// so they appear under their own names; the code is the same.
template <int M, typename R, int WV, int Tag = 0>
__global__ void __launch_bounds__(64 * WV) __attribute__((amdgpu_waves_per_eu(3)))
k_sweep_tb(Dev d, State<R> s, SweepLaunch a) {
    __shared__ double shm[SWEEP_SHM<M, WV>];
    const int nb = gridDim.x - 1;
    if (blockIdx.x == 0) {
        if (a.prev_nsw > 0 && !a.devfix && !s.ctl->done) sweep_test<M, R, WV>(d, s, a, shm);
        return;
    }
    b_sweep_tb<M, R, WV>(d, s, a, xcd_tile((int)blockIdx.x - 1, nb), shm);
}

// FP32 form: renormalise every link pair (b, l) by Knuth's two-sum, b' = fl(b + l) and
// l' = (b + l) - b' exactly, so the represented links do not change and the remainders
// the sweeps work on restart near zero.
template <typename R>
__device__ __forceinline__ void b_rebase(const Dev& d, const State<R>& s, int lcur, int tile) {
#pragma clang fp contract(off)
    if constexpr (!std::is_same<R, float>::value) return;  // FP64 keeps no bases
    int i, j;
    node_of(d, tile, i, j);
    if (i >= d.nx || j >= d.ny) return;
    int64_t n = at(d, i, j);
    const int64_t P = d.plane;
    R* l = s.l[lcur];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        R b = s.lb[q * P + n], r = l[q * P + n];
        R hi = b + r;
        R bv = hi - b;
        R lo = (b - (hi - bv)) + (r - bv);
        s.lb[q * P + n] = hi;
        l[q * P + n] = lo;
    }
}
template <typename R>
__global__ void __launch_bounds__(NT) k_rebase(Dev d, State<R> s, int lcur, int gate) {
    if (gate && s.ctl->done) return;  // inside a loop: only while it runs
    b_rebase<R>(d, s, lcur, xcd_tile(blockIdx.x, gridDim.x));
}

// FP32 form, after every renormalisation and with the solve's 1/tau_l: the launch constants
// of the sweeps.  With link = b + l and phi_B the bases' moment, the collided link is
// A(l) + C with A the collision of the remainders on their own moment and
// C = b - omega (b - w phi_B); a remainder pulled from node y therefore gains
// D = C(y) - b(x), and at an electrode the anti-bounce-back remainder is D - A with
// D = 2 w phi_wall - C_opp(x) - b(x).  D is formed in FP64 and rounded once (a small
// difference of nearly equal bases).
// node(dx, dy, b, om): the four link bases b[0..3] and omega of node (i + dx, j + dy), for the
// four neighbours and the node itself.
template <typename R, typename NodeAt>
__device__ __forceinline__ void sweep_consts(const Dev& d, const State<R>& s, int i, int j, NodeAt&& node) {
    const int64_t P = d.plane;
    auto cq = [&](int q, int dx, int dy) -> double {  // C of link q at node (i + dx, j + dy)
        double b[4], om;
        node(dx, dy, b, om);
        const double pb = ((b[0] + b[1]) + (b[2] + b[3])) * INV_1MW0;
        const double bq = b[q - 1];
        return bq - om * (bq - LWA * pb);
    };
    double b[4], om;
    node(0, 0, b, om);
    const int64_t n = at(d, i, j);
    const double d1 = cq(1, -1, 0) - b[0];
    const double d3 = cq(3, 1, 0) - b[2];
    const double d2 = (j == 0 ? 2.0 * LWA * d.phi_bot - cq(4, 0, 0) : cq(2, 0, -1)) - b[1];
    const double d4 = (j == d.ny - 1 ? 2.0 * LWA * d.phi_top - cq(2, 0, 0) : cq(4, 0, 1)) - b[3];
    s.dl[n] = R(d1);
    s.dl[P + n] = R(d2);
    s.dl[2 * P + n] = R(d3);
    s.dl[3 * P + n] = R(d4);
    s.pbp[n] = R(((b[0] + b[1]) + (b[2] + b[3])) * INV_1MW0);
}
template <typename R>
__device__ __forceinline__ void b_sweep_prep(const Dev& d, const State<R>& s, int tile) {
    if constexpr (!std::is_same<R, float>::value) return;  // FP64 keeps no bases
    int i, j;
    node_of(d, tile, i, j);
    if (i >= d.nx || j >= d.ny) return;
    const int64_t P = d.plane;
    sweep_consts<R>(d, s, i, j, [&](int dx, int dy, double (&b)[4], double& om) {
        const int64_t m = at(d, wrapx(i + dx, d.nx), j + dy);
#pragma unroll
        for (int q = 0; q < 4; q++) b[q] = s.lb[q * P + m];
        om = s.oml[m];
    });
}
// FP32 form, at a solve's start: the renormalisation of k_rebase and the constants of
// k_sweep_prep in one pass.  The renormalised pairs go to the idle potential buffer lnew and the
// other base set s.lbx, so the pairs of the neighbours this pass reads stay those of buffer
// lcur; a node's renormalised base is its pair's rounded sum (the high part of the two-sum),
// staged with omega for the tile and its one-node ring in LDS, so the constants are those of
// the two passes, bitwise.
template <typename R>
struct RebasedNode {
    R b[4];
    R om;
};
template <typename R>
__device__ __forceinline__ void b_rebase_prep(const Dev& d, const State<R>& s, int lcur, int lnew, int tile) {
#pragma clang fp contract(off)
    if constexpr (!std::is_same<R, float>::value) return;  // FP64 keeps no bases
    __shared__ RebasedNode<R> ring[RN];
    const int64_t P = d.plane;
    const R* l = s.l[lcur];
    stage_ring(d, tile, ring, [&](int64_t m) {
        RebasedNode<R> v;
#pragma unroll
        for (int q = 0; q < 4; q++) v.b[q] = s.lb[q * P + m] + l[q * P + m];
        v.om = s.oml[m];
        return v;
    });
    int i, j;
    node_of(d, tile, i, j);
    if (i >= d.nx || j >= d.ny) return;
    const int64_t n = at(d, i, j);
    R* lo_out = s.l[lnew];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        R b = s.lb[q * P + n], r = l[q * P + n];
        R hi = b + r;
        R bv = hi - b;
        R lo = (b - (hi - bv)) + (r - bv);
        s.lbx[q * P + n] = hi;
        lo_out[q * P + n] = lo;
    }
    const int me = ring_self();
    sweep_consts<R>(d, s, i, j, [&](int dx, int dy, double (&b)[4], double& om) {
        const RebasedNode<R>& v = ring[ring_from(me, -dx, -dy)];
#pragma unroll
        for (int q = 0; q < 4; q++) b[q] = v.b[q];
        om = v.om;
    });
}
template <typename R>
__global__ void __launch_bounds__(NT) k_rebase_prep(Dev d, State<R> s, int lcur, int lnew) {
    b_rebase_prep<R>(d, s, lcur, lnew, xcd_tile(blockIdx.x, gridDim.x));
}
template <typename R>
__global__ void __launch_bounds__(NT) k_sweep_prep(Dev d, State<R> s, int gate) {
    if (gate && s.ctl->done) return;
    b_sweep_prep<R>(d, s, xcd_tile(blockIdx.x, gridDim.x));
}

// The convergence test of the last launch of a batch (same rule as above), in two launches:
// TEST_RANGES blocks at most sum contiguous ranges of the tile partials (k_sweep_test_part),
// then one block adds the range sums in order and decides (k_sweep_test; parts = 0: it sums
// every tile itself).  256 threads a block: a 1024-thread block spent about 10 us on the
// reduction itself, at any tile count.
constexpr int TEST_NT = 256;
// LDS doubles of a test workgroup: the parked sums (M <= 8), else the range sums of
// k_sweep_test, which outnumber the per-wave sums of block_sums_waves
template <int M>
constexpr int TEST_SHM = M > 8 ? 2 * M * TEST_RANGES : 2 * M * TEST_NT + 2 * M;
__host__ __device__ constexpr int64_t part_test(int nb, int nbt) { return part_total(nb, nbt); }
template <int M, typename R>
__global__ void __launch_bounds__(TEST_NT) k_sweep_test_part(Dev d, State<R> s, SweepLaunch a) {
    __shared__ double sh[TEST_SHM<M>];
    if (s.ctl->done) return;
    const int nbt = d.tbx * d.tby, parts = gridDim.x;
    const int b0 = (int)((int64_t)nbt * blockIdx.x / parts), b1 = (int)((int64_t)nbt * (blockIdx.x + 1) / parts);
    double acc[2 * M];
    sweep_sums<M, R, TEST_NT / 64, 4>(d, s, a, sh, b0, b1, acc);
    if (threadIdx.x != 0) return;
    double* out = s.partials + part_test(part_nb(d), nbt) + (int64_t)blockIdx.x * 2 * SW_MAXM;
#pragma unroll
    for (int m = 0; m < 2 * M; m++) out[m] = acc[m];
}
// The outcome is published to host memory the caller polls: two 64-bit words, each carrying
// the sequence number `seq` in its upper half (the host waits for both), written with
// system-scope atomic stores: word 0 = count, word 1 = fix_launch << 7 | fix_n << 2 |
// conv << 1 | done.
template <int M, typename R>
__global__ void __launch_bounds__(TEST_NT) k_sweep_test(Dev d, State<R> s, SweepLaunch a, int parts,
                                                        unsigned long long* word, unsigned seq) {
    static_assert(2 * M * TEST_RANGES <= TEST_SHM<M>, "the range sums fit the block's shared array");
    __shared__ double sh[TEST_SHM<M>];
    if (!s.ctl->done) {
        if (parts > 0) {
            // range sums in block order: every thread stages a share of them in LDS (one
            // memory latency), then thread v adds value v of every range
            __shared__ double tot[2 * M];
            const double* in = s.partials + part_test(part_nb(d), d.tbx * d.tby);
            for (int k = threadIdx.x; k < parts * 2 * M; k += TEST_NT)
                sh[k] = in[(int64_t)(k / (2 * M)) * 2 * SW_MAXM + k % (2 * M)];
            __syncthreads();
            if (threadIdx.x < 2 * M) {
                double t = 0.0;
                for (int b = 0; b < parts; b++) t += sh[b * 2 * M + threadIdx.x];
                tot[threadIdx.x] = t;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                double acc[2 * M];
#pragma unroll
                for (int m = 0; m < 2 * M; m++) acc[m] = tot[m];
                sweep_decide<M>(s.ctl, a, acc);
            }
        } else {
            sweep_test<M, R, TEST_NT / 64, 4>(d, s, a, sh);
        }
    }
    if (threadIdx.x != 0 || !word) return;  // no word: a test inside a batch, nothing published
    // a.src: the solve's first buffer; the stage kernels that follow a loop read its final
    // buffer from here
    if (s.ctl->done) {
        const int src = stop_src(s.ctl, a.src);
        s.ctl->final_buf = stop_recompute(s.ctl) ? (src + 2) % 3 : (src + 1) % 3;
    }
    const Ctl* c = s.ctl;
    const unsigned long long hi = (unsigned long long)seq << 32;
    const unsigned long long w0 = hi | (unsigned)c->count;
    const unsigned long long w1 = hi | ((unsigned)c->fix_launch << 7 | (unsigned)c->fix_n << 2 |
                                        (unsigned)c->conv << 1 | (unsigned)c->done);
    __hip_atomic_store(&word[0], w0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&word[1], w1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void k_ctl_reset(Ctl* c, double tol, int min_sweeps, int max_sweeps) {
    ctl_reset(c, tol, min_sweeps, max_sweeps);
}

// ---------------------------------------------------------------------------
// Stage 3, the flow step: surface tension (Eqs. (3)-(5)) and electric force (Eq. (14)) from
// psi^{n+1}; S = rho mdot + u . grad(rho) (Eq. (24)); the collision inputs of h (rho, F~,
// F + rho f_solid, 1/tau_h); h pulled and collided at its source with bounce-back at the
// walls; u* (Eq. (25)), u (Eq. (26) with u_s = 0) and p (Eq. (27)).
//
// The chain psi, f_s -> rho -> S -> collision inputs -> pulls reaches three nodes out, so a
// workgroup owns a strip of WX columns and a segment of d.hseg rows and walks down it WR rows
// per pass, each quantity kept in LDS in a small ring of rows:
//   psi^{n+1} (wetting ghost), f_s and rho (mirror ghost)   WX + 6 columns, 8 rows
//   p (mirror ghost), phi (Dirichlet ghost), epsilon, S      WX + 4 columns, 6 rows
//   collision inputs and F                                   WX + 2 columns, 6 rows
// Pass t (rows b .. b + 3) stages psi, f_s, rho three rows ahead (b + 3 ..), p, phi,
// epsilon and S two rows ahead, the collision inputs one row ahead, then streams rows b ..
// b + 3.  Rows behind the window are never evaluated again, so besides the x halo only the
// first pass of a segment evaluates anything twice.  WX + 2 = 64: one wave per row of
// collision inputs.

template <typename R>
struct HWin {
    R ps[8 * WQ], fs[8 * WQ], rho[8 * WQ];  // row y at slot (y - jb) & 7
    R p[6 * WS], ph[6 * WS], S[6 * WS];     // row y at slot (y - jb) mod 6
    K eps[6 * WS];
    R in[10][6 * WE];  // collision inputs, member by member (HIn order), rows as p
    R Fx[6 * WE], Fy[6 * WE];
    int col[WQ];  // grid column of window column c (x wrapped)
};
template <typename R>
__device__ __forceinline__ HIn<R> hin_at(const HWin<R>& L, int o) {
    return HIn<R>{L.in[0][o], L.in[1][o], L.in[2][o], L.in[3][o], L.in[4][o],
                  L.in[5][o], L.in[6][o], L.in[7][o], L.in[8][o], L.in[9][o]};
}
template <typename R>
__device__ __forceinline__ void hin_put(HWin<R>& L, int o, const HIn<R>& a) {
    L.in[0][o] = a.p; L.in[1][o] = a.rho; L.in[2][o] = a.ux; L.in[3][o] = a.uy; L.in[4][o] = a.S;
    L.in[5][o] = a.Ftx; L.in[6][o] = a.Fty; L.in[7][o] = a.Gx; L.in[8][o] = a.Gy; L.in[9][o] = a.om;
}

// S = rho mdot + u . grad(rho) at a node with mass source md and velocity (ux, uy); vr is
// the density around it.
template <typename R>
__device__ __forceinline__ R source_S(R md, R ux, R uy, const R (&vr)[3][3]) {
    K w[3][3];
    to_k(vr, w);
    K grx, gry, dum;
    grad_lap<K>(w, grx, gry, dum);
    return R(w[1][1] * (K)md + (K)ux * grx + (K)uy * gry);
}

// F = F_s + F_e at a node from psi, epsilon and phi around it.
template <typename R>
__device__ __forceinline__ void h_force(const Dev& d, const R (&vp)[3][3], const K (&ve)[3][3],
                                        const R (&vph_r)[3][3], K& FxOut, K& FyOut) {
    K wp[3][3], vph[3][3];
    to_k(vp, wp);
    to_k(vph_r, vph);
    K gx, gy, lap;
    grad_lap<K>(wp, gx, gy, lap);
    K ps = wp[1][1];
    K mu = 4.0 * d.beta * ps * (ps - 1.0) * (ps - 0.5) - d.kappa * lap;
    K Fx = mu * gx, Fy = mu * gy;
    K gpx, gpy, lphi, gex, gey, dum;
    grad_lap<K>(vph, gpx, gpy, lphi);
    grad_lap<K>(ve, gex, gey, dum);
    K eps = ve[1][1];
    K Ex = -gpx, Ey = -gpy;
    K qv = -(gex * gpx + gey * gpy + eps * lphi);
    K E2 = Ex * Ex + Ey * Ey;
    Fx += qv * Ex - 0.5 * E2 * gex;
    Fy += qv * Ey - 0.5 * E2 * gey;
    FxOut = Fx;
    FyOut = Fy;
}

// Collision inputs of h at a node: vr, vpr and vs are rho, p and S around it; ps and fs its
// own psi and f_s, (ux, uy) its velocity, (usx, usy) its u* of the previous step, F its force.
template <typename R>
__device__ __forceinline__ HIn<R> h_inputs(const Dev& d, R ps, R fs, const R (&vr)[3][3], const R (&vpr_r)[3][3],
                                           const R (&vs)[3][3], R ux, R uy, R usx, R usy, K Fx, K Fy) {
    K wr[3][3], vpr[3][3], ws[3][3];
    to_k(vr, wr);
    to_k(vpr_r, vpr);
    to_k(vs, ws);
    K grx, gry, gpx, gpy, gsx = 0.0, gsy = 0.0, dum;
    grad_lap<K>(wr, grx, gry, dum);
    grad_lap<K>(vpr, gpx, gpy, dum);
    if (d.readings & 1u) grad_lap<K>(ws, gsx, gsy, dum);
    const R rho_r = vr[1][1];
    K rho = wr[1][1];
    K fsn = (K)fs;
    R mu = mix<R>(d.mu_s, d.mu_l, d.mu_g, ps, fs);
    return HIn<R>{vpr_r[1][1],
                  rho_r,
                  ux,
                  uy,
                  vs[1][1],
                  R(Fx - gpx + CS2 * grx + CS2 * gsx),
                  R(Fy - gpy + CS2 * gry + CS2 * gsy),
                  R(Fx + rho * (fsn * (0.0 - (K)usx))),
                  R(Fy + rho * (fsn * (0.0 - (K)usy))),
                  R(1) / (mu / (rho_r * R(CS2)) + R(0.5))};
}

// h pulled and collided at its source, bounce-back at the walls; u* (Eq. (25)), u (Eq. (26)
// with u_s = 0), p (Eq. (27)).  hv[q]: the stored value the pull of direction q reads (h_q at
// the source, or h_opp(q) at this node where the source is beyond a wall; FP16 storage: the
// binary16 value, not yet scaled and offset); nbr(q): collision inputs of the source (a node
// inside the grid); (Fx, Fy) and fsn: this node's force and solid fraction.  Returns the
// largest binary16-stored deviation (FP16 storage) or 0.
template <typename R, bool H, typename NB>
__device__ __forceinline__ float h_stream_at(const Dev& d, const State<R>& s, int sp, int i, int j,
                                             const HIn<R>& self, NB&& nbr, const R (&hv)[9], H16Scales hs,
                                             R Fx, R Fy, R fsn) {
    const int64_t n = at(d, i, j);
    R* hdst = s.h[sp ^ 1];
    R sx = R(0), sy = R(0), s0 = R(0);
    R vals[H ? 9 : 1];
#pragma unroll
    for (int q = 0; q < 9; q++) {
        int jj = j - QY[q];
        R val;
        if (jj < 0 || jj >= d.ny) {
            int o = QOPP[q];
            R raw = hv[q];
            if constexpr (H) raw = h_rest<R>(o, self.p) + raw * hs.inv;
            val = coll_h<R>(o, raw, self);
        } else {
            const HIn<R> a = nbr(q);
            R raw = hv[q];
            if constexpr (H) raw = h_rest<R>(q, a.p) + raw * hs.inv;
            val = coll_h<R>(q, raw, a);
        }
        if constexpr (H) vals[q] = val;
        else hdst[q * d.plane + n] = val;
        sx += R(QX[q]) * val;
        sy += R(QY[q]) * val;
        if (q) s0 += val;
    }
    R rho = self.rho;
    R ax = (sx + R(0.5) * Fx) / rho;
    R ay = (sy + R(0.5) * Fy) / rho;
    s.usx[sp ^ 1][n] = ax;
    s.usy[sp ^ 1][n] = ay;
    R ux = ax + R(0.5) * fsn * (R(0) - ax);
    R uy = ay + R(0.5) * fsn * (R(0) - ay);
    s.ux[sp ^ 1][n] = ux;
    s.uy[sp ^ 1][n] = uy;
    R uF = self.ux * self.Ftx + self.uy * self.Fty;
    R R0 = R(W0) * (self.S - R(3) * uF);
    R uu = ux * ux + uy * uy;
    R s0u = R(W0) * (R(-1.5) * uu);
    const R pn = R(CS2 / (1.0 - W0)) * (s0 + R(0.5) * self.S + (R(1) / self.om) * R0 + rho * s0u);
    s.p[sp ^ 1][n] = pn;
    float mx = 0.f;
    if constexpr (H) {
        // deviations from the equilibrium of the pressure stored beside them
#pragma unroll
        for (int q = 0; q < 9; q++) {
            const float dv = vals[q] - h_rest<R>(q, pn);
            mx = fmaxf(mx, fabsf(dv));
            h16_put((half_t*)hdst, q * d.plane + n, dv, hs.sc);
        }
    }
    return mx;
}

// Rows of pass t of a window (segment rows [jb, je)): psi, f_s, rho rows [qlo, qhi); p, phi,
// epsilon, S rows [plo, phi); collision inputs rows [elo, ehi); streamed rows b .. b + 3.
struct HPass {
    int b, qlo, qhi, plo, phi, elo, ehi;
};
__device__ __forceinline__ HPass h_pass(const Dev& d, int jb, int je, int t) {
    HPass a;
    a.b = jb + WR * t;
    a.qlo = max(t < 0 ? jb - 3 : a.b + 3, -1);
    a.qhi = min(min(a.b + 7, je + 3), d.ny + 1);
    a.plo = max(t < 0 ? jb - 2 : a.b + 2, -1);
    a.phi = min(min(a.b + 6, je + 2), d.ny + 1);
    a.elo = max(t < 0 ? jb - 1 : a.b + 1, 0);
    a.ehi = min(min(a.b + 5, je + 1), d.ny);
    return a;
}

// The global reads of one pass's staging, held in registers from the pass before: psi and
// f_s (Q items), p and phi (P items), mdot and u (the S items), u and u* (this wave's row of
// collision inputs).  Each thread holds at most two items of each kind (items k = threadIdx.x
// and threadIdx.x + NT; a pass has at most 6 * WQ < 2 * NT Q items and 4 * WS P items).
template <typename R>
struct HFetch {
    R qps[2], qfs[2], pp[2], pph[2], smd[2], sux[2], suy[2];
    R eux, euy, eusx, eusy;
};

template <typename R, bool H = false>
__device__ __forceinline__ void b_h_fused(const Dev& d, const State<R>& s, int sp, int lcur, int tile) {
    static_assert(6 * WQ <= 2 * NT && WR * WS <= 2 * NT, "two staging items per thread at most");
    __shared__ HWin<R> L;
    const int i0 = (tile % d.hx) * WX, jb = (tile / d.hx) * d.hseg;
    const int je = min(jb + d.hseg, d.ny);
    for (int c = threadIdx.x; c < WQ; c += NT) L.col[c] = wrap_col(i0 - 3 + c, d.nx);
    H16Scales hs{};
    if constexpr (H) hs = h16_scales(s.ctl, PS_H, sp, tile == 0);
    float mx = 0.f;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const R* psi = s.psi[sp ^ 1];
    const R* fs = s.fs[sp];
    const R* pr = s.p[sp];
    const R* ph = s.phi[lcur];
    const R* ux = s.ux[sp];
    const R* uy = s.uy[sp];
    const R* md = s.md[sp];
    const R* hsrc = s.h[sp];
    auto q8 = [&](int y) { return ((y - jb + 8) & 7) * WQ; };
    auto r6 = [&](int y) { return (y - jb + 6) % 6; };
    __syncthreads();  // L.col
    // issue the global reads of pass t's staging
    auto fetch = [&](int t, HFetch<R>& f) {
        const HPass a = h_pass(d, jb, je, t);
        const int nq = (a.qhi - a.qlo) * WQ, np = (a.phi - a.plo) * WS;
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int k = threadIdx.x + u * NT;
            if (k < nq) {
                const int64_t m = at(d, L.col[k % WQ], clamp_row(a.qlo + k / WQ, d.ny));
                f.qps[u] = psi[m];
                f.qfs[u] = fs[m];
            }
            if (k < np) {
                const int y = a.plo + k / WS;
                const int64_t m = at(d, L.col[k % WS + 1], clamp_row(y, d.ny));
                f.pp[u] = pr[m];
                f.pph[u] = ph[m];
                if (y >= 0 && y < d.ny) {
                    f.smd[u] = md[m];
                    f.sux[u] = ux[m];
                    f.suy[u] = uy[m];
                }
            }
        }
        const int ye = a.elo + wv;
        if (ye < a.ehi) {
            const int64_t m = at(d, L.col[lane + 2], ye);
            f.eux = ux[m];
            f.euy = uy[m];
            f.eusx = s.usx[sp][m];
            f.eusy = s.usy[sp][m];
        }
    };
    HFetch<R> f;
    fetch(-1, f);
    // Pass -1 fills the rings for pass 0: psi, f_s, rho rows jb - 3 .., p, phi, epsilon, S rows
    // jb - 2 .., collision inputs rows jb - 1 and jb.  Pass t >= 0 (b = jb + 4 t) adds psi, f_s,
    // rho rows b + 3 .. b + 6, p, phi, epsilon, S rows b + 2 .. b + 5 and collision inputs rows
    // b + 1 .. b + 4, then streams rows b .. b + 3.  Rows past what the segment's last row needs,
    // and beyond the ghost rows, are skipped.  Global reads are issued a phase ahead of the
    // arithmetic that waits for them: a pass's staging reads during the previous pass's
    // streaming, its pulls of h before its collision inputs are evaluated.
    for (int t = -1;; t++) {
        const HPass a = h_pass(d, jb, je, t);
        const int b = a.b;
        if (b >= je) break;
        const int nq = (a.qhi - a.qlo) * WQ, np = (a.phi - a.plo) * WS;
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int k = threadIdx.x + u * NT;
            if (k < nq) {
                const int y = a.qlo + k / WQ, c = k % WQ;
                const R pv = ghost_fix<GWET, R>(f.qps[u], d, y), fv = ghost_fix<GMIRROR, R>(f.qfs[u], d, y);
                const int o = q8(y) + c;
                L.ps[o] = pv;
                L.fs[o] = fv;
                L.rho[o] = mix<R>(d.rho_s, d.rho_l, d.rho_g, pv, fv);
            }
            if (k < np) {
                const int y = a.plo + k / WS, c = k % WS;
                const int o = r6(y) * WS + c;
                L.p[o] = ghost_fix<GMIRROR, R>(f.pp[u], d, y);
                L.ph[o] = ghost_fix<GPHI, R>(f.pph[u], d, y);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int k = threadIdx.x + u * NT;
            if (k >= np) break;
            const int y = a.plo + k / WS, c = k % WS;
            const int o = r6(y) * WS + c, qo = q8(y) + c + 1;
            L.eps[o] = mix<K>(d.eps_s, d.eps_l, d.eps_g, (K)L.ps[qo], (K)L.fs[qo]);
            if (y >= 0 && y < d.ny) {
                R vr[3][3];
                rows3(L.rho + q8(y - 1), L.rho + q8(y), L.rho + q8(y + 1), c + 1, vr);
                L.S[o] = source_S<R>(f.smd[u], f.sux[u], f.suy[u], vr);
            }
        }
        __syncthreads();
        // this pass's streamed node (row b + wv, column i0 + lane): its solid fraction and the
        // nine values its pulls read
        const int j = b + wv, i = i0 + lane;
        const bool gv = t >= 0 && j < je && lane < WX && i < d.nx;
        R fsn = R(0);
        R hv[9];
        if (gv) {
            fsn = L.fs[q8(j) + lane + 3];
            const int64_t n = at(d, i, j);
#pragma unroll
            for (int q = 0; q < 9; q++) {
                const int jj = j - QY[q];
                const int64_t k = (jj < 0 || jj >= d.ny) ? QOPP[q] * d.plane + n
                                                         : q * d.plane + at(d, wrapx(i - QX[q], d.nx), jj);
                if constexpr (H) hv[q] = (R)((const half_t*)hsrc)[k];
                else hv[q] = hsrc[k];
            }
        }
        const int ye = a.elo + wv;
        if (ye < a.ehi) {
            const int c = lane;
            R vp[3][3], vr[3][3], vpr[3][3], vph[3][3], vs[3][3];
            K ve[3][3];
            rows3(L.ps + q8(ye - 1), L.ps + q8(ye), L.ps + q8(ye + 1), c + 2, vp);
            rows3(L.rho + q8(ye - 1), L.rho + q8(ye), L.rho + q8(ye + 1), c + 2, vr);
            const int sm = r6(ye - 1) * WS, s0 = r6(ye) * WS, sq = r6(ye + 1) * WS;
            rows3(L.p + sm, L.p + s0, L.p + sq, c + 1, vpr);
            rows3(L.ph + sm, L.ph + s0, L.ph + sq, c + 1, vph);
            rows3(L.eps + sm, L.eps + s0, L.eps + sq, c + 1, ve);
            // S beyond a wall: the mirror ghost is the wall row's own value
            const int ys = ye > 0 ? sm : s0, yn = ye < d.ny - 1 ? sq : s0;
            rows3(L.S + ys, L.S + s0, L.S + yn, c + 1, vs);
            K Fx, Fy;
            h_force<R>(d, vp, ve, vph, Fx, Fy);
            const int o = r6(ye) * WE + c;
            hin_put(L, o, h_inputs<R>(d, vp[1][1], L.fs[q8(ye) + c + 2], vr, vpr, vs, f.eux, f.euy, f.eusx,
                                      f.eusy, Fx, Fy));
            L.Fx[o] = R(Fx);
            L.Fy[o] = R(Fy);
        }
        __syncthreads();
        if (b + WR < je) fetch(t + 1, f);
        if (gv) {
            const int c = lane + 1;
            const int rm = r6(j - 1) * WE, r0 = r6(j) * WE, rp = r6(j + 1) * WE;
            // source of direction q: (i - cx, j - cy)
            auto nbr = [&](int q) -> HIn<R> {
                const int row = QY[q] > 0 ? rm : (QY[q] < 0 ? rp : r0);
                return hin_at(L, row + c - QX[q]);
            };
            const float m = h_stream_at<R, H>(d, s, sp, i, j, hin_at(L, r0 + c), nbr, hv, hs, L.Fx[r0 + c],
                                              L.Fy[r0 + c], fsn);
            mx = fmaxf(mx, m);
        }
    }
    if constexpr (H) h16_note_max(&s.ctl->hmax[PS_H][sp ^ 1], mx);
}
// Stage kernels queued behind a potential loop before the host knows its outcome are gated:
// with lcur < 0 the kernel runs only if the loop has ended (else the host queues it again
// once it has) and takes the final potential buffer from the control block.
// Waves per SIMD the flow step is compiled for: three in FP32 (its 33 KB of LDS would allow
// four; the registers alone give two, and three spill 6 of them: 406 against 420 us at
// 4096 x 2048), two otherwise (FP16 storage would spill 18 and run 15% slower at three; the
// FP64 window's 63 KB of LDS holds it at two workgroups per CU anyway).
template <typename R, bool H>
constexpr int H_WAVES = (sizeof(R) == 4 && !H) ? 3 : 2;
template <typename R, bool H = false>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(H_WAVES<R, H>)))
k_h_fused(Dev d, State<R> s, int sp, int lcur) {
    if (lcur < 0) {
        if (!s.ctl->done) return;
        lcur = s.ctl->final_buf;
    }
    b_h_fused<R, H>(d, s, sp, lcur, xcd_tile(blockIdx.x, gridDim.x));
}

template <typename R>
__device__ __forceinline__ GIn<R> g_inputs(const Dev& d, R ps, R fsn, R T, R Hn, R ux, R uy, R md) {
    R C = mix<R>(d.C_s, d.C_l, d.C_g, ps, fsn);
    R k = mix<R>(d.k_s, d.k_l, d.k_g, ps, fsn);
    return GIn<R>{Hn, T, C, ux, uy, R(1) / (k / (R(d.Cref) * R(CS2)) + R(0.5)), C * T * md};
}

// Stage 4: g pulled and collided at its source; substrate anti-bounce-back at T_w,
// adiabatic top; H^{n+1} = sum g + Q/2 (Eq. (30)); Eq. (7) gives T, f_l; new f_s
// and mdot.  Per-block FP64 liquid volume for the freezing-time detector.
// One pass over a window (see AX): the collision inputs of g one row ahead (AE columns, from
// point values read during the previous pass's streaming), then the streaming of rows
// b .. b + 3 with the pulls read before the inputs are evaluated.
template <typename R>
struct GWin {
    R in[7][6 * AE];  // collision inputs member by member (GIn order), row y at slot slot6(y, jb)
    int col[AS];
};
template <typename R>
__device__ __forceinline__ GIn<R> gin_at(const GWin<R>& L, int o) {
    return GIn<R>{L.in[0][o], L.in[1][o], L.in[2][o], L.in[3][o], L.in[4][o], L.in[5][o], L.in[6][o]};
}
template <typename R, bool H = false>
__device__ __forceinline__ void b_g_stream(const Dev& d, const State<R>& s, int sp, int tile) {
    __shared__ GWin<R> L;
    const int i0 = (tile % d.gx) * AX, jb = (tile / d.gx) * d.hseg;
    const int je = min(jb + d.hseg, d.ny);
    for (int c = threadIdx.x; c < AS; c += NT) L.col[c] = wrap_col(i0 - 2 + c, d.nx);
    H16Scales hs{};
    if constexpr (H) hs = h16_scales(s.ctl, PS_G, sp, tile == 0);
    float mx = 0.f;
    double vl = 0.0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const R* gsrc = s.g[sp];
    R* gdst = s.g[sp ^ 1];
    const R Cref = R(d.Cref);
    constexpr bool based = std::is_same<R, float>::value;
    __syncthreads();  // L.col
    struct Fetch {
        R ps[2], fs[2], T[2], Hn[2], ux[2], uy[2], md[2];
    } f;
    auto fetch = [&](int t) {
        const SPass a = s_pass(d, jb, je, t);
        const int ne = (a.ehi - a.elo) * AE;
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int k = threadIdx.x + u * NT;
            if (k < ne) {
                const int64_t m = at(d, L.col[k % AE + 1], a.elo + k / AE);
                f.ps[u] = s.psi[sp ^ 1][m];
                f.fs[u] = s.fs[sp][m];
                f.T[u] = s.T[sp][m];
                f.Hn[u] = s.H[sp][m];
                f.ux[u] = s.ux[sp ^ 1][m];
                f.uy[u] = s.uy[sp ^ 1][m];
                f.md[u] = s.md[sp][m];
            }
        }
    };
    fetch(-1);
    for (int t = -1;; t++) {
        const SPass a = s_pass(d, jb, je, t);
        const int b = a.b;
        if (b >= je) break;
        // this pass's streamed node (row b + wv, column i0 + lane): the nine values its pulls
        // read and its own fields
        const int j = b + wv, i = i0 + lane;
        const bool gv = t >= 0 && j < je && i < d.nx;
        R hv[9], ps1 = R(0), hb = R(0), ps0 = R(0), ux0 = R(0), uy0 = R(0), fs0 = R(0);
        if (gv) {
            const int64_t n = at(d, i, j);
#pragma unroll
            for (int q = 0; q < 9; q++) {
                const int jj = j - QY[q];
                const int64_t k = (jj < 0 || jj >= d.ny) ? QOPP[q] * d.plane + n
                                                         : q * d.plane + at(d, wrapx(i - QX[q], d.nx), jj);
                if constexpr (H) hv[q] = (R)((const half_t*)gsrc)[k];
                else hv[q] = gsrc[k];
            }
            ps1 = s.psi[sp ^ 1][n];
            if (based) hb = s.hb[n];
            ps0 = s.psi[sp][n];
            ux0 = s.ux[sp][n];
            uy0 = s.uy[sp][n];
            fs0 = s.fs[sp][n];
        }
        const int ne = (a.ehi - a.elo) * AE;
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int k = threadIdx.x + u * NT;
            if (k >= ne) break;
            const GIn<R> g = g_inputs<R>(d, f.ps[u], f.fs[u], f.T[u], f.Hn[u], f.ux[u], f.uy[u], f.md[u]);
            const int o = slot6(a.elo + k / AE, jb) * AE + k % AE;
            L.in[0][o] = g.H;
            L.in[1][o] = g.T;
            L.in[2][o] = g.C;
            L.in[3][o] = g.ux;
            L.in[4][o] = g.uy;
            L.in[5][o] = g.om;
            L.in[6][o] = g.Q;
        }
        __syncthreads();
        if (b + WR < je) fetch(t + 1);
        if (gv) {
            const int64_t n = at(d, i, j);
            const int c = lane + 1;
            const int rm = slot6(j - 1, jb) * AE, r0 = slot6(j, jb) * AE, rp = slot6(j + 1, jb) * AE;
            const GIn<R> self = gin_at(L, r0 + c);
            R sum = R(0), g0 = R(0);
            R vals[H ? 9 : 1];
#pragma unroll
            for (int q = 0; q < 9; q++) {
                int jj = j - QY[q];
                int o = QOPP[q];
                R val;
                if (jj < 0) {
                    R raw = hv[q];
                    if constexpr (H) raw = g_rest<R>(o, self.H, self.T, Cref) + raw * hs.inv;
                    val = -coll_g<R>(o, raw, self, Cref) + R(2.0 * QW[q] * d.Cref * d.T_w);
                } else if (jj >= d.ny) {
                    R raw = hv[q];
                    if constexpr (H) raw = g_rest<R>(o, self.H, self.T, Cref) + raw * hs.inv;
                    val = coll_g<R>(o, raw, self, Cref);
                } else {
                    const int row = QY[q] > 0 ? rm : (QY[q] < 0 ? rp : r0);
                    const GIn<R> an = gin_at(L, row + c - QX[q]);
                    R raw = hv[q];
                    if constexpr (H) raw = g_rest<R>(q, an.H, an.T, Cref) + raw * hs.inv;
                    val = coll_g<R>(q, raw, an, Cref);
                }
                if (q == 0) g0 = val;
                if constexpr (H) vals[q] = val;
                else gdst[q * d.plane + n] = val;
                sum += val;
            }
            R Hn = sum + R(0.5) * self.Q;
            R T, fl;
            invert<R>(d, Hn, hb, ps1, T, fl);
            if (based) {
                // move the base to the new psi: rest link and H re-expressed exactly (the
                // product is rounded on its own, as in the inversion)
#pragma clang fp contract(off)
                R hn = clamp01(ps1) * R(d.Lvol);
                R shift = hb - hn;
                if constexpr (H) vals[0] = g0 + shift;
                else gdst[n] = g0 + shift;
                Hn = Hn + shift;
                s.hb[n] = hn;
            }
            if constexpr (H) {
                // deviations from the equilibrium of the H and T stored beside them
#pragma unroll
                for (int q = 0; q < 9; q++) {
                    const float dv = vals[q] - g_rest<R>(q, Hn, T, Cref);
                    mx = fmaxf(mx, fabsf(dv));
                    h16_put((half_t*)gdst, q * d.plane + n, dv, hs.sc);
                }
            }
            R fsn = clamp01(ps1) * (R(1) - fl);
            // (psi u)^n for the next step's A (its readers in this step have all run)
            s.pux[n] = ps0 * ux0;
            s.puy[n] = ps0 * uy0;
            s.H[sp ^ 1][n] = Hn;
            s.T[sp ^ 1][n] = T;
            s.fl[n] = fl;
            s.md[sp ^ 1][n] = R(d.shrink) * (fsn - fs0);
            s.fs[sp ^ 1][n] = fsn;
            vl += (double)(clamp01(ps1) * fl);
        }
        __syncthreads();  // the next pass's inputs go into the rows this pass read
    }
    if constexpr (H) h16_note_max(&s.ctl->hmax[PS_G][sp ^ 1], mx);
    __shared__ double sh[NT / 64];
    double bv = block_sum(vl, sh);
    if (threadIdx.x == 0) s.partials[part_vl(part_nb(d)) + tile] = bv;
}

template <typename R, bool H = false>
__global__ void __launch_bounds__(NT) k_g_stream(Dev d, State<R> s, int sp, int gate) {
    if (gate && !s.ctl->done) return;
    b_g_stream<R, H>(d, s, sp, xcd_tile(blockIdx.x, gridDim.x));
}

// One block: liquid volume of the new state (block partials in order).  mode 1 records
// V_l0 after initialisation; mode 0 advances the step counter and runs the freezing-time
// detector: t_fre is the first step with V_l <= 1% of V_l0, interpolated linearly.
__global__ void __launch_bounds__(NT) k_vl_finalize(Dev d, const double* partials, Ctl* c, int mode, int gate) {
    __shared__ double sh[NT / 64];
    if (gate && !c->done) return;
    vl_finalize_body(d, partials, c, mode, sh);
}

// Per-window liquid volume of the initial state (finalized by k_vl_finalize, mode 1), over the
// windows of the g stage so that every liquid-volume sum has the same blocks.
template <typename R>
__device__ __forceinline__ void b_vl0(const Dev& d, const State<R>& s, int tile) {
    const int i0 = (tile % d.gx) * AX, jb = (tile / d.gx) * d.hseg;
    const int je = min(jb + d.hseg, d.ny);
    const int lane = threadIdx.x & 63, i = i0 + lane;
    double vl = 0.0;
    if (i < d.nx)
        for (int j = jb + (threadIdx.x >> 6); j < je; j += WR) {
            const int64_t n = at(d, i, j);
            vl += (double)(clamp01(s.psi[0][n]) * s.fl[n]);
        }
    __shared__ double sh[NT / 64];
    double bv = block_sum(vl, sh);
    if (threadIdx.x == 0) s.partials[part_vl(part_nb(d)) + tile] = bv;
}
template <typename R>
__global__ void __launch_bounds__(NT) k_vl0(Dev d, State<R> s) {
    b_vl0<R>(d, s, xcd_tile(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// Diagnostics: per-block FP64 sums, max |u| and a non-finite count; k_diag_finalize
// adds them in block order and scans the centre column for the droplet height
// (psi = 1/2) and the freezing front (f_l = 1/2).
// A field value in FP64 with the ghost rule G applied in FP64 (x already wrapped).
template <int G, typename R>
__device__ __forceinline__ double ghosted_d(const R* __restrict__ f, const Dev& d, int i, int j) {
    if (j < 0) {
        const double b = (double)f[i];
        if (G == GWET) return b + d.wet * b * (1.0 - b);
        if (G == GPHI) return 2.0 * d.phi_bot - b;
        return b;
    }
    if (j >= d.ny) {
        const double t = (double)f[at(d, i, d.ny - 1)];
        return G == GPHI ? 2.0 * d.phi_top - t : t;
    }
    return (double)f[at(d, i, j)];
}

// Operator residual of the potential equation at node (i, j): div(sigma grad phi) written with
// Eq. (36) as grad(sigma).grad(phi) + sigma lap(phi) (the discrete form q_v takes for eps),
// sigma mixed by Eq. (1) from psi (wetting ghost) and f_s (mirrored); *ramp: the same for the
// linear electrode ramp (Dirichlet ghosts) with this sigma.  FP64 throughout.
template <typename R>
__device__ __forceinline__ double op_residual(const Dev& d, const R* psi, const R* fs, const R* phi, int i, int j,
                                              double* ramp) {
    const int im = wrapx(i - 1, d.nx), ip = wrapx(i + 1, d.nx);
    const int cols[3] = {im, i, ip};
    double vs[3][3], vp[3][3], vl[3][3];
#pragma unroll
    for (int dy = -1; dy <= 1; dy++) {
        const int jj = j + dy;
        const double lin = jj < 0 ? 2.0 * d.phi_bot - phi_lin(d, 0)
                           : (jj >= d.ny ? 2.0 * d.phi_top - phi_lin(d, d.ny - 1) : phi_lin(d, jj));
#pragma unroll
        for (int dx = 0; dx < 3; dx++) {
            const double ps = ghosted_d<GWET, R>(psi, d, cols[dx], jj);
            const double f = ghosted_d<GMIRROR, R>(fs, d, cols[dx], jj);
            vs[dy + 1][dx] = mix<double>(d.sig_s, d.sig_l, d.sig_g, ps, f);
            vp[dy + 1][dx] = ghosted_d<GPHI, R>(phi, d, cols[dx], jj);
            vl[dy + 1][dx] = lin;
        }
    }
    double gsx, gsy, dum, gpx, gpy, lap, glx, gly, llap;
    grad_lap<double>(vs, gsx, gsy, dum);
    grad_lap<double>(vp, gpx, gpy, lap);
    grad_lap<double>(vl, glx, gly, llap);
    const double sg = vs[1][1];
    *ramp = gsx * glx + gsy * gly + sg * llap;
    return gsx * gpx + gsy * gpy + sg * lap;
}

template <typename R, bool H = false>
__device__ __forceinline__ void b_diag(const Dev& d, const State<R>& s, int sp, int lcur, int tile) {
    int i, j;
    node_of(d, tile, i, j);
    double v[DIAG_N] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (i < d.nx && j < d.ny) {
        int64_t n = at(d, i, j);
        double ps = s.psi[sp][n];
        double fl = s.fl[n];
        double ux = s.ux[sp][n], uy = s.uy[sp][n];
        v[0] = ps;
        double sf = 0.0, sg = 0.0;
        for (int q = 0; q < 9; q++) {
            if constexpr (H) {
                const float fi = ldexpf(1.f, -s.ctl->hexp[PS_F][sp]), gi = ldexpf(1.f, -s.ctl->hexp[PS_G][sp]);
                const R psn = s.psi[sp][n];
                sf += (double)h16_get((const half_t*)s.f[sp], q * d.plane + n, f_rest<R>(q, psn), fi);
                sg += (double)h16_get((const half_t*)s.g[sp], q * d.plane + n,
                                      g_rest<R>(q, s.H[sp][n], s.T[sp][n], R(d.Cref)), gi);
            } else {
                // FP32: f held as deviations from w_i psi
                sf += (double)s.f[sp][q * d.plane + n] +
                      (std::is_same<R, float>::value ? (double)f_rest<R>(q, s.psi[sp][n]) : 0.0);
                sg += (double)s.g[sp][q * d.plane + n];
            }
        }
        v[1] = sf;
        v[2] = std::is_same<R, float>::value ? sg + (double)s.hb[n] : sg;
        v[3] = (double)clamp01(s.psi[sp][n]) * fl;
        v[4] = s.fs[sp][n];
        v[5] = sqrt(ux * ux + uy * uy);
        double chk = ps + ux + uy + (double)s.p[sp][n] + (double)s.T[sp][n] + (double)s.phi[lcur][n];
        v[6] = isfinite(chk) ? 0.0 : 1.0;
        double rr;
        const double ro = op_residual<R>(d, s.psi[sp], s.fs[sp], s.phi[lcur], i, j, &rr);
        v[7] = ro * ro;
        v[8] = rr * rr;
    }
    __shared__ double sh[NT / 64];
    double r[DIAG_N];
    for (int k = 0; k < 5; k++) r[k] = block_sum(v[k], sh);
    r[5] = block_max(v[5], sh);
    for (int k = 6; k < DIAG_N; k++) r[k] = block_sum(v[k], sh);
    if (threadIdx.x == 0) {
        double* pw = s.partials + part_diag(part_nb(d)) + DIAG_N * (int64_t)tile;
        for (int k = 0; k < DIAG_N; k++) pw[k] = r[k];
    }
}
template <typename R, bool H = false>
__global__ void __launch_bounds__(NT) k_diag(Dev d, State<R> s, int sp, int lcur) {
    b_diag<R, H>(d, s, sp, lcur, xcd_tile(blockIdx.x, gridDim.x));
}

template <typename R>
__global__ void __launch_bounds__(NT) k_diag_finalize(Dev d, State<R> s, int sp) {
    __shared__ double sh[NT / 64];
    int nb = d.gx * d.gy;
    const double* pv = s.partials + part_diag(part_nb(d));
    double a[DIAG_N] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = threadIdx.x; k < nb; k += NT) {
        for (int m = 0; m < 5; m++) a[m] += pv[DIAG_N * k + m];
        a[5] = fmax(a[5], pv[DIAG_N * k + 5]);
        for (int m = 6; m < DIAG_N; m++) a[m] += pv[DIAG_N * k + m];
    }
    double out[DIAG_N];
    for (int m = 0; m < 5; m++) out[m] = block_sum(a[m], sh);
    out[5] = block_max(a[5], sh);
    for (int m = 6; m < DIAG_N; m++) out[m] = block_sum(a[m], sh);
    if (threadIdx.x != 0) return;
    Ctl* c = s.ctl;
    for (int m = 0; m < 6; m++) c->dsum[m] = out[m];
    c->nonfinite = out[6] > 0.0;
    c->op_res[0] = sqrt(out[7]);
    c->op_res[1] = sqrt(out[8]);
    const R* psi = s.psi[sp];
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
    if (psi[at(d, ic, 0)] >= R(0.5)) {
        front = height;
        for (int jj = 0; jj < d.ny && psi[at(d, ic, jj)] >= R(0.5); jj++) {
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

// ---------------------------------------------------------------------------
// Batched form: many cases of different grid sizes advanced together.  Each case keeps
// its own constants, state and control block; a table in device memory lists them with
// the first block of each case in the node grid and in the blocked-sweep grid.  One
// launch per stage covers every case: block b (XCD-ordered) finds its case by binary
// search and runs the same body as the single-case kernel on that case's tile b - first.

template <typename R>
struct BatchCase {
    Dev d;
    State<R> s;
};

__device__ __forceinline__ int find_case(const int* __restrict__ first, int ncases, int b) {
    int lo = 0, hi = ncases - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

#define LBM_BATCHED(name, body, ...)                                                        \
    template <typename R>                                                                   \
    __global__ void __launch_bounds__(NT) name(const BatchCase<R>* __restrict__ cases,      \
                                               const int* __restrict__ first, int ncases,  \
                                               int sp, const int* __restrict__ lcur) {     \
        int b = xcd_tile(blockIdx.x, gridDim.x);                                            \
        int c = find_case(first, ncases, b);                                                \
        const BatchCase<R>& bc = cases[c];                                                  \
        if (bc.s.ctl->frozen) return;                                                       \
        body<R>(bc.d, bc.s, ##__VA_ARGS__, b - first[c]);                                   \
    }

LBM_BATCHED(kb_oml, b_oml, sp)
LBM_BATCHED(kb_rebase, b_rebase, lcur[c])
LBM_BATCHED(kb_sweep_prep, b_sweep_prep)
LBM_BATCHED(kb_vl0, b_vl0)
#undef LBM_BATCHED

// The same for the stage bodies that also serve the FP16-storage form (H).
#define LBM_BATCHED_H(name, body, ...)                                                      \
    template <typename R, bool H = false>                                                   \
    __global__ void __launch_bounds__(NT) name(const BatchCase<R>* __restrict__ cases,      \
                                               const int* __restrict__ first, int ncases,  \
                                               int sp, const int* __restrict__ lcur) {     \
        int b = xcd_tile(blockIdx.x, gridDim.x);                                            \
        int c = find_case(first, ncases, b);                                                \
        const BatchCase<R>& bc = cases[c];                                                  \
        if (bc.s.ctl->frozen) return;                                                       \
        body<R, H>(bc.d, bc.s, ##__VA_ARGS__, b - first[c]);                                \
    }

LBM_BATCHED_H(kb_init, b_init)
LBM_BATCHED_H(kb_f_fused, b_f_fused, sp)
LBM_BATCHED_H(kb_h_fused, b_h_fused, sp, lcur[c])
LBM_BATCHED_H(kb_g_stream, b_g_stream, sp)
#undef LBM_BATCHED_H

// FP32 rebase of the cases whose potential loop is still running after launch t - 1 (their
// state is in buffer (lcur0 + t) mod 3).
template <typename R>
__global__ void __launch_bounds__(NT) kb_rebase_running(const BatchCase<R>* __restrict__ cases,
                                                        const int* __restrict__ first, int ncases,
                                                        const int* __restrict__ lcur0, int t) {
    int b = xcd_tile(blockIdx.x, gridDim.x);
    int c = find_case(first, ncases, b);
    const BatchCase<R>& bc = cases[c];
    if (bc.s.ctl->done || bc.s.ctl->frozen) return;
    b_rebase<R>(bc.d, bc.s, (lcur0[c] + t) % 3, b - first[c]);
}

// Launch t of a lockstep potential loop for one case: sweeps t*M+1 .. of that case, from
// the buffer the case's solve started in; the previous launch is the one to test.
template <int M>
__device__ __forceinline__ SweepLaunch lockstep_launch(const Ctl* c, int lcur0, int t) {
    SweepLaunch a{};
    a.k0 = t * M + 1;
    a.nsw = min(M, c->max_sweeps + 1 - a.k0);
    if (a.nsw < 0) a.nsw = 0;
    a.src = (lcur0 + t) % 3;
    a.dst = (a.src + 1) % 3;
    a.slot = t & 1;
    a.launch = t;
    if (t > 0) {
        a.prev_k0 = (t - 1) * M + 1;
        a.prev_nsw = min(M, c->max_sweeps + 1 - a.prev_k0);
        a.prev_slot = (t - 1) & 1;
    }
    return a;
}

template <int M, typename R, int WV>
__global__ void __launch_bounds__(64 * WV) __attribute__((amdgpu_waves_per_eu(3))) kb_sweep(const BatchCase<R>* __restrict__ cases, const int* __restrict__ first,
                                                    int ncases, const int* __restrict__ lcur0, int t,
                                                    const int* __restrict__ idx) {
    // The launch covers the ncases cases listed in idx (the loops still running when the
    // batch of launches was queued; first: their first sweep tiles in the launch).  The first
    // ncases blocks test each case's previous launch while the others sweep (as in the
    // single-case launch: dispatched first, the tests are off the critical path and a case
    // they end skips the blocks that start later).
    const int ntiles = gridDim.x - ncases;
    __shared__ double shm[SWEEP_SHM<M, WV>];
    if ((int)blockIdx.x < ncases) {
        const int c = idx[blockIdx.x];
        const BatchCase<R>& bc = cases[c];
        SweepLaunch a = lockstep_launch<M>(bc.s.ctl, lcur0[c], t);
        if (a.nsw > 0 && a.prev_nsw > 0 && !bc.s.ctl->done) sweep_test<M, R, WV>(bc.d, bc.s, a, shm);
        return;
    }
    int b = xcd_tile((int)blockIdx.x - ncases, ntiles);
    int cc = find_case(first, ncases, b);
    const int c = idx[cc];
    const BatchCase<R>& bc = cases[c];
    SweepLaunch a = lockstep_launch<M>(bc.s.ctl, lcur0[c], t);
    if (a.nsw == 0) return;
    b_sweep_tb<M, R, WV>(bc.d, bc.s, a, b - first[cc], shm);
}

// Recomputation of each finished case's last launch up to its final sweep (fix[c].nsw = 0:
// nothing to redo for that case).
template <int M, typename R, int WV>
__global__ void __launch_bounds__(64 * WV) __attribute__((amdgpu_waves_per_eu(3))) kb_sweep_fix(const BatchCase<R>* __restrict__ cases, const int* __restrict__ first,
                                                        int ncases, const SweepLaunch* __restrict__ fix) {
    int b = xcd_tile(blockIdx.x, gridDim.x);
    int c = find_case(first, ncases, b);
    __shared__ double shm[SWEEP_SHM<M, WV>];
    SweepLaunch a = fix[c];
    if (a.nsw == 0) return;
    const BatchCase<R>& bc = cases[c];
    b_sweep_tb<M, R, WV>(bc.d, bc.s, a, b - first[c], shm);
}

// One block per case: test the case's launch t (the last of a batch).
template <int M, typename R>
__global__ void __launch_bounds__(TEST_NT) kb_sweep_test(const BatchCase<R>* __restrict__ cases,
                                                         const int* __restrict__ lcur0, int t,
                                                         const int* __restrict__ idx) {
    __shared__ double sh[TEST_SHM<M>];
    const int c = idx[blockIdx.x];
    const BatchCase<R>& bc = cases[c];
    if (bc.s.ctl->done) return;
    SweepLaunch a = lockstep_launch<M>(bc.s.ctl, lcur0[c], t + 1);
    if (a.prev_nsw <= 0) return;
    sweep_test<M, R, TEST_NT / 64, 4>(bc.d, bc.s, a, sh);
}

template <typename R>
__global__ void kb_ctl_reset(const BatchCase<R>* __restrict__ cases, int ncases, const double* tol, int min_sweeps,
                             const int* max_sweeps) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncases) return;
    Ctl* ct = cases[c].s.ctl;
    ct->fix_launch = 0;
    ct->fix_n = 0;
    ct->fix_k0 = 0;
    ct->fix_nsw = 0;
    ct->done = ct->frozen;  // a frozen case takes no part in the loop
    ct->count = 0;
    ct->conv = ct->frozen;
    ct->resid = 0.0;
    ct->tol = tol[c];
    ct->min_sweeps = min_sweeps;
    ct->max_sweeps = max_sweeps[c];
}

// One block per case: the liquid volume of the case's new state (see k_vl_finalize).
template <typename R>
__global__ void __launch_bounds__(NT) kb_vl_finalize(const BatchCase<R>* __restrict__ cases, int mode) {
    __shared__ double sh[NT / 64];
    const BatchCase<R>& bc = cases[blockIdx.x];
    const Dev& d = bc.d;
    Ctl* c = bc.s.ctl;
    if (c->frozen) return;
    const int nb = d.gx * d.hy;  // one partial per window of the g stage
    const double* pv = bc.s.partials + part_vl(part_nb(d));
    double a = 0.0;
    for (int k = threadIdx.x; k < nb; k += NT) a += pv[k];
    a = block_sum(a, sh);
    if (threadIdx.x != 0) return;
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

// ---------------------------------------------------------------------------
// Learned warm start of the potential: coarse input maps, coarse target, and the seeding of
// the potential links.  Coarse cell (I, J) covers the fine nodes [I f, (I + 1) f) x
// [J f, (J + 1) f); coarse maps are NHWC with the x index fastest.

// Input maps averaged over a cell: clamped psi, ln(sigma / sigma_gas), ln(eps / eps_gas)
// with sigma and eps mixed by Eq. (1) (0 when the gas permittivity is 0), from psi of buffer
// psp and f_s of buffer fsp.
template <typename R>
__global__ void __launch_bounds__(NT) k_nn_features(Dev d, State<R> s, int psp, int fsp, int f,
                                                    float* __restrict__ x) {
    const int nxc = d.nx / f, nyc = d.ny / f;
    const int c = blockIdx.x * NT + threadIdx.x;
    if (c >= nxc * nyc) return;
    const int I = c % nxc, J = c / nxc;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int j = J * f; j < (J + 1) * f; j++)
        for (int i = I * f; i < (I + 1) * f; i++) {
            const int64_t n = at(d, i, j);
            const double ps = (double)s.psi[psp][n], fs = (double)s.fs[fsp][n];
            a0 += clamp01(ps);
            a1 += log(mix<double>(d.sig_s, d.sig_l, d.sig_g, ps, fs) / d.sig_g);
            if (d.eps_g > 0.0) a2 += log(mix<double>(d.eps_s, d.eps_l, d.eps_g, ps, fs) / d.eps_g);
        }
    const double inv = 1.0 / ((double)f * f);
    x[3 * (int64_t)c] = (float)(a0 * inv);
    x[3 * (int64_t)c + 1] = (float)(a1 * inv);
    x[3 * (int64_t)c + 2] = (float)(a2 * inv);
}

// Target: the cell average of (phi - ramp) / (phi_top - phi_bot).
template <typename R>
__global__ void __launch_bounds__(NT) k_nn_target(Dev d, State<R> s, int lcur, int f, float* __restrict__ t) {
    const int nxc = d.nx / f, nyc = d.ny / f;
    const int c = blockIdx.x * NT + threadIdx.x;
    if (c >= nxc * nyc) return;
    const int I = c % nxc, J = c / nxc;
    double a = 0.0;
    for (int j = J * f; j < (J + 1) * f; j++)
        for (int i = I * f; i < (I + 1) * f; i++) a += (double)s.phi[lcur][at(d, i, j)] - phi_lin(d, j);
    t[c] = (float)(a / ((double)f * f) / (d.phi_top - d.phi_bot));
}

// Seed: phi = ramp + (phi_top - phi_bot) * (bilinear interpolation of the coarse deviation at
// the node, cell-centred values, periodic in x, clamped in y); the four links of buffer lcur
// become their equilibria w_i phi (FP32: base/remainder pairs) and phi is written.
template <typename R>
__device__ __forceinline__ void b_nn_seed(const Dev& d, const State<R>& s, int lcur, int f,
                                          const float* __restrict__ yc, int tile) {
    int i, j;
    node_of(d, tile, i, j);
    if (i >= d.nx || j >= d.ny) return;
    const int nxc = d.nx / f, nyc = d.ny / f;
    // The sweeps conserve the moving links' sum at every node and carry it to a neighbour of
    // the other colour of the checkerboard (a wall returns it negated to the same node), so
    // Q = sum over nodes of (-1)^(i+j) (l1 + l2 + l3 + l4) changes sign every sweep whatever
    // 1/tau_l is: a mode that never decays, and a seed with Q != 0 leaves a relative change
    // that never meets the stopping rule.  The seed is therefore evaluated once per pair of
    // nodes (2k, 2k+1) of a row, at the pair's centre: the two nodes get identical links
    // and Q = 0 exactly for even nx (for odd nx the periodic rows have no such mode).
    const double X = ((i & ~1) + 1.0) / f - 0.5, Y = (j + 0.5) / f - 0.5;
    const int i0 = (int)floor(X), j0 = (int)floor(Y);
    const double fx = X - i0, fy = Y - j0;
    const int ia = (i0 % nxc + nxc) % nxc, ib = (ia + 1) % nxc;
    const int ja = j0 < 0 ? 0 : (j0 > nyc - 1 ? nyc - 1 : j0);
    const int jb = j0 + 1 > nyc - 1 ? nyc - 1 : (j0 + 1 < 0 ? 0 : j0 + 1);
    const double v = (1.0 - fy) * ((1.0 - fx) * yc[ja * nxc + ia] + fx * yc[ja * nxc + ib]) +
                     fy * ((1.0 - fx) * yc[jb * nxc + ia] + fx * yc[jb * nxc + ib]);
    const double phi = phi_lin(d, j) + (d.phi_top - d.phi_bot) * v;
    const double leq = LWA * phi;
    const int64_t n = at(d, i, j);
    constexpr bool based = std::is_same<R, float>::value;
    R base = based ? R(leq) : R(0);
    R l = R(leq - (double)base);
#pragma unroll
    for (int q = 0; q < 4; q++) {
        s.l[lcur][q * d.plane + n] = l;
        if (based) s.lb[q * d.plane + n] = base;
    }
    s.phi[lcur][n] = based ? R(phi) : (l + l + l + l) * R(INV_1MW0);
}
template <typename R>
__global__ void __launch_bounds__(NT) k_nn_seed(Dev d, State<R> s, int lcur, int f, const float* __restrict__ yc) {
    b_nn_seed<R>(d, s, lcur, f, yc, xcd_tile(blockIdx.x, gridDim.x));
}

}  // namespace lbm

