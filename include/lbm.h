/*
 * lbm.h -- C ABI of the MI355X (gfx950) electrofreezing lattice Boltzmann library.
 *
 * The library advances the coupled phase-field lattice Boltzmann method of
 * Huang, Li, Che, Chai, Wang, Shi, "Freezing dynamics of wetting droplet under a
 * uniform electric field" (arXiv:2410.06657) on one GPU:
 *   - f, D2Q9: conservative Allen-Cahn phase field psi with the freezing volume
 *     source (Sec. 3.1, Eqs. (15)-(20));
 *   - h, D2Q9: pressure and velocity with the mass source and the diffuse solid
 *     force (Sec. 3.2, Eqs. (21)-(27));
 *   - g, D2Q9: total (volumetric) enthalpy, temperature and solid fraction
 *     (Sec. 3.3, Eqs. (28)-(30), inversion Eq. (7));
 *   - l, D2Q5: electric potential of the leaky-dielectric model, swept to
 *     convergence inside every time step (Sec. 3.4, Eqs. (31)-(34), Algorithm 1);
 *   - the coupling terms: isotropic gradients and Laplacians (Eq. (36)), surface
 *     tension (Eqs. (3)-(5)), electric force (Eq. (14)), property mixing (Eq. (1)).
 *
 * Grid and layout.  Nodes (i, j), 0 <= i < nx (periodic), 0 <= j < ny, at x = i,
 * y = j.  Half-way walls at y = -1/2 (cooled substrate, lower electrode) and
 * y = ny - 1/2 (upper electrode).  Host arrays exchanged through this ABI are
 * FP64, row-major [j][i] for fields and [q][j][i] for populations (q in the
 * order rest, E, N, W, S, NE, NW, SW, SE for D2Q9 and rest, E, N, W, S for D2Q5).
 * Temperatures are measured from the melting point (T_m = 0).
 *
 * Memory ownership.  The caller allocates one device workspace of
 * lbm_workspace_bytes() bytes and owns it and the stream; the library carves
 * every device array out of that workspace and never allocates or frees device
 * memory.  It owns the small host-side handle (and a few bytes of pinned host
 * memory for flag read-back).  Host pointers passed in are borrowed for the
 * duration of the call only.  A handle is used by one host thread at a time.
 *
 * Errors.  Every function returns LBM_OK (0) or a negative code; no C++
 * exception crosses the ABI.  lbm_strerror() names a code; after LBM_EHIP the
 * HIP error string of the last failing call is kept in the handle and returned
 * by lbm_last_error().
 */
#ifndef LBM_ABI_INCLUDED
#define LBM_ABI_INCLUDED

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_EINVAL (-1)     /* bad argument or parameter value */
#define LBM_ENOCONV (-2)    /* potential sweeps hit the cap before the stopping test */
#define LBM_ENONFINITE (-3) /* NaN or Inf found by the diagnostics */
#define LBM_EHIP (-4)       /* a HIP runtime call failed */
#define LBM_ESTATE (-5)     /* call out of order (e.g. step before init) */
#define LBM_ESPACE (-6)     /* workspace smaller than lbm_workspace_bytes() */

/* Arithmetic and storage (lbm_params.precision).  FP64: every population and field in
   double.  FP32: populations, fields and the populations' arithmetic in float: the
   phase-field populations are stored as deviations from w_i psi of their node and collided,
   streamed and summed in that deviation form; the enthalpy rest link and H are stored
   relative to the node's latent heat psi rho_s L; the D2Q5 links are FP32 base/remainder
   pairs (their increments are below an FP32 ulp of the raw values).  The coupling terms
   (gradients, Laplacians, normals, chemical potential, forces, sources) are evaluated in FP64
   from the stored fields in every form, as are the potential residual, the liquid and solid
   volume sums, the freezing-time detector and the front search.  FP32_FP16STORE: the
   FP32 form with the f, h and g populations stored in binary16 as deviations from the
   zero-velocity equilibria of their nodes' stored moments (Eqs. (18), (22), (29)), each set
   scaled by a power of two that follows its largest deviation one step earlier; the
   potential links keep the FP32 base/remainder pairs (a binary16 link could not resolve the
   1e-8 stopping rule); each case of a batch keeps its own scales.  lbm_get_pop decodes the binary16 sets on the host, lbm_set_pop returns LBM_EINVAL for f, h
   and g (a write would have to be encoded against the running scales).  Because its populations are stored
   relative to the node's stored psi, p, H and T, lbm_set_field of one of those fields also
   moves that node's f, h or g populations by the change of their zero-velocity equilibria;
   in the FP32 form the same holds for psi and f (in FP64 the populations stay as they are).
   The ABI always exchanges raw FP64 values. */
#define LBM_FP64 0
#define LBM_FP32 1
#define LBM_FP32_FP16STORE 2

/* Reading switches (bits of lbm_params.readings). */
#define LBM_R_GRAD_S 1u /* F~ of Eq. (24) contains c_s^2 grad(S) (the printed "div S") */

/* Case parameters, lattice units.  Properties of the three phases are mixed by
   Eq. (1) with psi clamped to [0, 1]. */
typedef struct lbm_params {
    int nx, ny;
    int precision;              /* LBM_FP64, LBM_FP32 or LBM_FP32_FP16STORE */
    double W, M, gamma;         /* interface width, mobility (Eq. (2a)), surface tension */
    double rho_l, rho_g, rho_s; /* densities */
    double mu_l, mu_g, mu_s;    /* dynamic viscosities */
    double cp_l, cp_g, cp_s;    /* specific heat per unit mass */
    double k_l, k_g, k_s;       /* thermal conductivities */
    double latent;              /* latent heat per unit mass */
    double T_w, T_g;            /* substrate temperature, initial temperature */
    double eps_l, eps_g, eps_s; /* permittivities */
    double sig_l, sig_g, sig_s; /* electric conductivities */
    double phi_top, phi_bot;    /* electrode potentials */
    double theta_deg;           /* contact angle at the substrate */
    int shape;                  /* initial interface: 0 disc (R0, xc, yc), 1 layer of thickness h0 */
    double R0, xc, yc, h0;
    double poisson_tol;         /* relative sweep-to-sweep change that ends a solve; < 0: fixed count */
    int poisson_max_sweeps;     /* cap per solve */
    unsigned readings;          /* LBM_R_* bits */
    int sweep_block;            /* potential sweeps per kernel launch: 1, 2, 4, 8 or 16 (0: 8;
                                   16 only with sweep_waves 8).  A launch keeps every sweep's
                                   residual, so the stopping sweep is the same for any value. */
    int sweep_waves;            /* 64-lane waves per sweep workgroup, 4 or 8 (0: 4): the
                                   region a workgroup sweeps is 64 x (8 * sweep_waves) nodes.
                                   Results do not depend on it (nor on sweep_block). */
    int skip_initial_solve;     /* 1: lbm_init leaves the linear-ramp potential unsolved (sweep
                                   log entry 0) for the caller to seed (lbm_warm_start) and
                                   solve (lbm_solve_potential); 0: solve as in Algorithm 1.
                                   A batch takes it when every case has the same value (then
                                   lbm_batch_warm_start, lbm_batch_solve_potential). */
    int stage_rows;             /* rows of the segment each workgroup of the f, flow and g
                                   stages walks down its strip: a multiple of 4 from 4 to 512
                                   (0: 32, lowered in steps of 4 while the flow launch would
                                   have fewer than 2048 workgroups).  A launch-shape choice
                                   (lbm_autotune picks one): every field is the same for any
                                   value; only the order in which the liquid-volume partial
                                   sums are added, hence the last bits of V_l, depends on it. */
} lbm_params;

/* Scalar fields for lbm_get_field / lbm_set_field. */
enum {
    LBM_PSI = 0, LBM_UX, LBM_UY, LBM_USX, LBM_USY, LBM_P, LBM_T, LBM_H,
    LBM_FS, LBM_MDOT, LBM_PSIU_X, LBM_PSIU_Y, LBM_PHI, LBM_FL,
    LBM_NFIELDS
};
/* Population sets for lbm_get_pop / lbm_set_pop. */
enum { LBM_POP_F = 0, LBM_POP_H = 1, LBM_POP_G = 2, LBM_POP_L = 3 };

/* Global output of Algorithm 1, all reductions in FP64. */
typedef struct lbm_diag {
    long long step;
    double sum_psi, sum_f, sum_g; /* sums of psi and of the f and g populations */
    double V_l, V_s;              /* sum of psi f_l (liquid volume) and of f_s */
    double front_y;               /* f_l = 1/2 crossing on column nx/2, from the wall */
    double height;                /* psi = 1/2 crossing on column nx/2, from the wall */
    double max_u;                 /* max |u| */
    double resid;                 /* relative change at the last potential sweep */
    int sweeps;                   /* sweeps of the last potential solve */
    int noconv;                   /* solves inside lbm_step that hit the cap */
    double t_fre;                 /* freezing step: V_l first <= 1% of V_l0, interpolated; -1 if not yet */
    double V_l0;                  /* V_l at initialisation */
    int nonfinite;                /* 1 if psi, u, p, T or phi holds NaN/Inf */
    /* Operator residual of the potential equation div(sigma grad phi) = 0 (Sec. 2), written
       with the isotropic stencils of Eq. (36) as grad(sigma).grad(phi) + sigma lap(phi) (the
       discrete form the free charge of Eq. (14) takes for eps), sigma mixed by Eq. (1) from the
       current psi and f_s: its L2 norm over the grid for the current phi (op_resid) and for the
       linear electrode ramp with the same sigma (op_resid_ramp, where a solve starts; 0 for a
       uniform sigma).  The LB sweeps converge to their own discretisation of the interface
       conditions, so op_resid / op_resid_ramp levels off near a few percent on a W = 4
       interface instead of reaching 0; it shows gross non-convergence, the relative change
       (resid) the stopping rule. */
    double op_resid, op_resid_ramp;
    int init_converged;           /* 1 if lbm_init's potential solve met the stopping rule */
} lbm_diag;

typedef struct lbm_handle lbm_handle;

/* Bytes of device workspace needed by lbm_init for these parameters.
   LBM_EINVAL on bad parameters (tau <= 1/2 cannot occur: every relaxation time
   is 1/2 plus a positive transport coefficient, so positivity is what is checked). */
int lbm_workspace_bytes(const lbm_params* p, size_t* bytes);

/* The launch shapes a handle of these parameters takes, defaults resolved: potential sweeps
   per launch, waves per sweep workgroup and stage segment rows.  Host only; LBM_EINVAL on bad
   parameters or a null output. */
int lbm_launch_shapes(const lbm_params* p, int* sweep_block, int* sweep_waves, int* stage_rows);

/* Initialise (Algorithm 1, first block): psi from the tanh profile of the initial
   shape, u = u* = p = 0, T = T_g in fully liquid drops, phi a linear ramp between
   the electrodes, every population at its equilibrium (Eqs. (18), (22), (29), (32)),
   then one potential solve (at least two sweeps: a first sweep of equilibrium
   populations leaves a linear ramp unchanged).  `workspace` is a device pointer
   to at least lbm_workspace_bytes() bytes, 256-byte aligned; `stream` is a
   hipStream_t (NULL = the null stream).  Work is queued on the stream; the call
   returns after the initial solve has ended (it reads the loop's outcome).  If that solve
   reached poisson_max_sweeps before the stopping rule, lbm_init returns LBM_ENOCONV and
   still sets *out to a valid handle (lbm_diag.init_converged = 0); the caller decides
   whether to go on (lbm_solve_potential can continue the solve).  On any other error *out
   is left unset. */
int lbm_init(const lbm_params* p, void* workspace, size_t bytes, void* stream,
             lbm_handle** out);

/* n full time steps of Algorithm 1 in the order f (collide, stream, bounce-back,
   wetting) -> psi, rho, F_s -> potential swept to convergence -> phi, F_e ->
   h (collide, stream, bounce-back) -> u, p -> g (collide, stream, substrate at T_w)
   -> T, f_l, f_s.  Kernels run on the handle's stream; the host reads the
   potential's convergence flag once per batch of sweeps, and the rest of the step is
   queued behind each batch's test before that read (it runs only once the loop has
   ended), so the call returns with the last step's h and g stages possibly still
   running.  The last step's liquid volume and freezing-time detector are folded in by
   the next step's first kernel, or by any call that reads the control block
   (lbm_diagnostics, lbm_run_until_frozen, lbm_checkpoint).  A solve that hits the
   sweep cap leaves a valid state and is counted in lbm_diag.noconv. */
int lbm_step(lbm_handle* h, int n);

/* Sweep the potential (Eqs. (31)-(34)) with the current psi and f_s until the
   relative change ||phi^k - phi^{k-1}||_2 / ||phi^k||_2 <= tol (tol < 0: exactly
   max_sweeps sweeps).  Returns the sweep count and the last relative change;
   LBM_ENOCONV if the cap was reached first (the state stays valid). */
int lbm_solve_potential(lbm_handle* h, double tol, int max_sweeps, int* sweeps,
                        double* resid);

/* FP64 reductions of the current state into *out; synchronises the stream. */
int lbm_diagnostics(lbm_handle* h, lbm_diag* out);

/* Copy one field (nx*ny doubles) or one population set (nq*nx*ny doubles) between
   the device state and a host array; synchronise the stream.  nq is 9 for f, h, g
   and 4 for l: the D2Q5 rest link relaxes towards (w_0 - 1) phi but never enters
   phi (Eq. (34) sums links 1-4 only) nor the other links' collision, so it is
   not kept. */
int lbm_get_field(lbm_handle* h, int field, double* dst);
int lbm_set_field(lbm_handle* h, int field, const double* src);
int lbm_get_pop(lbm_handle* h, int set, double* dst);
int lbm_set_pop(lbm_handle* h, int set, const double* src);

/* One field as nx*ny FP64 values, row-major [j][i], into device memory `dst` (caller-owned,
   at least nx*ny*8 bytes): the same raw values lbm_get_field returns (bases added in the FP32
   forms), written by a kernel queued on the handle's stream; asynchronous, no host copy. */
int lbm_get_field_device(lbm_handle* h, int field, double* dst);

/* Sweep counts of every potential solve since lbm_init (index 0 = initial solve);
   copies min(count, cap) entries, *count gets the total. */
int lbm_sweep_log(lbm_handle* h, int* dst, int cap, int* count);

/* Step until the freezing time is detected (R30: t_fre > 0 after a step) or max_steps steps,
   testing every check_every steps (so up to check_every - 1 steps may follow the freezing
   step); *steps_done gets the steps taken.  t_fre itself comes from lbm_diagnostics. */
int lbm_run_until_frozen(lbm_handle* h, int max_steps, int check_every, int* steps_done);

/* Checkpoint: the whole state of a handle (every plane of the workspace, the control block,
   buffer indices, step counter and sweep log) as one host image.  With host == NULL only
   *bytes is set (the image size, which grows with the sweep log); else *bytes must be at
   least that size (LBM_ESPACE otherwise) and receives it.  Restore takes an image written by
   a handle of the same grid, precision and launch shape (LBM_EINVAL otherwise) and continues
   bitwise as the original would have.  Both synchronise the stream; host memory is the
   caller's. */
int lbm_checkpoint(lbm_handle* h, void* host, size_t* bytes);
int lbm_restore(lbm_handle* h, const void* host, size_t bytes);

/* Measurement: launch exactly n potential sweeps (Eqs. (31)-(34), the step's inner
   loop, in the launch configuration lbm_step uses: the first workgroup of each launch
   also evaluates the previous launch's residuals, but the loop never stops early) on
   the handle's stream, bracketed by HIP events; *ms gets the elapsed GPU time.  The
   state advances by n sweeps.  Synchronises the stream. */
int lbm_time_sweeps(lbm_handle* h, int n, float* ms);

/* Measurement: each kernel of the step outside the potential sweeps (Algorithm 1's f, h and g
   updates and their coupling terms; lbm_stage_name(k) names kernel k) launched n times back to
   back on the current state, bracketed by HIP events on the handle's stream; ms[k] gets the
   average duration of kernel k.  The kernels also rewrite the single-buffered planes a step
   carries into the next one (u*, psi u of the previous step, the FP32 enthalpy base), so the
   handle is left in LBM_ESTATE: every later call but lbm_destroy, lbm_restore and the
   measurement calls returns LBM_ESTATE until lbm_restore loads an image.  With ms == NULL only
   *nstages is set and nothing runs; cap must be at least *nstages.  Synchronises the stream. */
int lbm_time_stages(lbm_handle* h, int n, float* ms, int cap, int* nstages);
const char* lbm_stage_name(int k);

/* Measurement (no part of the method): the HBM rate a plain streaming kernel reaches on this
   GPU, as a reference beside the published peak for the rooflines.  Copies `bytes` from the
   device buffer src to the device buffer dst (both 16-byte aligned, bytes a positive multiple
   of 16; the buffers must not overlap) reps times back to back on `stream` with 16-byte loads
   and stores, bracketed by HIP events; *ms gets the average duration of one copy.  LBM_EINVAL
   on bad arguments.  Synchronises the stream. */
int lbm_time_copy(void* dst, const void* src, size_t bytes, void* stream, int reps, float* ms);

/* Autotuner of the launch shapes for one grid size and precision; the shapes change no
   field, only speed.  (1) Potential sweeps (sweeps per launch x waves per workgroup): every
   candidate in {2, 4, 8} x {4, 8} is initialised in the caller's device workspace
   (`workspace`, 256-byte aligned, at least lbm_autotune_workspace_bytes() bytes; its
   contents are overwritten; the library allocates nothing), then `launches` launches of it
   are timed twice on `stream` (the faster pass counts).  (2) Stage segments (stage_rows):
   the default of lbm_params.stage_rows = 0 and those of 8, 16, 32, 64 and 128 rows below the
   grid's height, each timed as the f, flow and g stages, `launches` launches of each, twice.
   In both, the default (8 sweeps x 4 waves; stage_rows = 0's height, candidate 0) is kept
   unless the fastest candidate beats it by more than 3%, so near ties do not flip the choice
   from run to run.  Results are cached
   per (nx, ny, precision) for the life of the process; flags & LBM_TUNE_FORCE re-times (a
   cached answer needs no workspace: pass NULL).  Other fields of *p only shape the timed
   state.  LBM_ESPACE if the workspace is smaller than needed.  Synchronises the stream. */
#define LBM_TUNE_FORCE 1
#define LBM_TUNE_MAXCAND 8
typedef struct {
    int sweep_block, sweep_waves;          /* the fastest sweep shape */
    int cached;                            /* 1: taken from the cache */
    int ncand;
    int cand_block[LBM_TUNE_MAXCAND];
    int cand_waves[LBM_TUNE_MAXCAND];
    float us_per_sweep[LBM_TUNE_MAXCAND];  /* measured time per sweep */
    int stage_rows;                        /* the fastest stage segment */
    int nrows;
    int cand_rows[LBM_TUNE_MAXCAND];
    float us_per_step_stages[LBM_TUNE_MAXCAND];  /* f + flow + g stage time per step */
} lbm_tune;
int lbm_autotune_workspace_bytes(const lbm_params* p, size_t* bytes);
int lbm_autotune(const lbm_params* p, void* workspace, size_t bytes, void* stream, int launches, int flags,
                 lbm_tune* out);

/* Release the handle (not the workspace, which the caller owns). */
int lbm_destroy(lbm_handle* h);

/* ---- Batched form: many independent cases of different grid sizes ------------------
   Every case is one run of the method above (Algorithm 1 with its own parameters and
   state), but each stage is one kernel launch covering the tiles of all cases, the
   stages outside the potential loop are replayed from HIP graphs (when the stream is not
   the null stream), and the potential loops of all cases run in lockstep launches in
   which cases that have converged exit at once.  All cases share `precision` and
   `sweep_block`.  The caller owns one workspace of lbm_batch_workspace_bytes() bytes
   (256-byte aligned) and the stream; the library allocates no device memory. */
typedef struct lbm_batch lbm_batch;

int lbm_batch_workspace_bytes(int ncases, const lbm_params* cases, size_t* bytes);
/* Initialise every case as lbm_init does (initial potential solves in lockstep). */
int lbm_batch_init(int ncases, const lbm_params* cases, void* workspace, size_t bytes,
                   void* stream, lbm_batch** out);
/* n time steps of every case. */
int lbm_batch_step(lbm_batch* b, int n);
/* Step the batch until every case has frozen (R30) or max_steps steps.  A case stops
   advancing right after the step in which its freezing time is detected: its workgroups exit
   at once in every later launch, its state, sweep log and step count stay those of that step
   (bitwise the single-case run stopped there), and the others continue.  Reads the control
   blocks after every step; *steps_done gets the batch steps taken. */
int lbm_batch_run_until_frozen(lbm_batch* b, int max_steps, int* steps_done);

/* FP64 diagnostics of every case into per_case[0..ncases-1]; synchronises. */
int lbm_batch_diagnostics(lbm_batch* b, lbm_diag* per_case);
/* One field of case c as nx_c*ny_c FP64 values; synchronises. */
int lbm_batch_get_field(lbm_batch* b, int c, int field, double* dst);
/* Sweep counts of case c's potential solves since init (see lbm_sweep_log). */
int lbm_batch_sweep_log(lbm_batch* b, int c, int* dst, int cap, int* count);
int lbm_batch_destroy(lbm_batch* b);

const char* lbm_strerror(int code);
const char* lbm_last_error(const lbm_handle* h);

/* ---- Learned warm start of the potential ------------------------------------------
   A network maps coarse maps of the state to the coarse deviation of the potential from the
   linear electrode ramp; its prediction seeds the potential links, after which the plain
   sweeps of Eqs. (31)-(34) run to the same stopping rule (they, not the network, decide the
   result).  The
   network: six 3x3 convolutions, 3 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1 channels, dilations
   1, 2, 4, 8, 4, 1, tanh between layers, zero padding; FP16 weights and activations with
   FP32 accumulation on the matrix cores; FP32 master parameters and Adam (beta 0.9, 0.999,
   eps 1e-8).  Coarse maps are FP32, NHWC (x fastest): input 3 maps per pixel (psi clamped to
   [0, 1], ln(sigma / sigma_gas), ln(eps / eps_gas), cell averages with sigma and eps mixed by
   Eq. (1)), output 1 map ((phi - ramp) / (phi_top - phi_bot), cell average).  Coarse cell
   (I, J) covers fine nodes [I f, (I+1) f) x [J f, (J+1) f); nx and ny must be multiples of
   the factor f.

   Parameter order (lbm_nn_param_count floats): for each layer l = 0..5 the weights
   [tap = 3 ky + kx][out 0..31][in 0..cin-1] (cin = 8 for layer 0, else 32; tap offset
   ((kx - 1) d, (ky - 1) d)), then the 6 x 32 biases.  Entries that are padding (inputs 3..7
   of layer 0, outputs 1..31 of layer 5) are held at zero. */
typedef struct lbm_nn lbm_nn;

int lbm_nn_param_count(int* count);
/* Device workspace for activations of up to max_pixels coarse pixels per call (images x
   height x width); caller-owned, 256-byte aligned. */
int lbm_nn_workspace_bytes(long long max_pixels, size_t* bytes);
/* Glorot-uniform initial weights from SplitMix64(seed), zero biases; kernels run on
   `stream`.  Synchronises the stream. */
int lbm_nn_init(void* workspace, size_t bytes, long long max_pixels, unsigned long long seed, void* stream,
                lbm_nn** out);
/* Host FP32 parameters in the order above; set also resets the Adam state. */
int lbm_nn_set_params(lbm_nn* nn, const float* host);
int lbm_nn_get_params(lbm_nn* nn, float* host);
/* x: device FP32 (n, h, w, 3); y: device FP32 (n, h, w).  Asynchronous on the stream. */
int lbm_nn_forward(lbm_nn* nn, const float* x, float* y, int n, int h, int w);
/* Gradient of L = sum over pixels of (y - t)^2 with respect to every parameter (host FP32,
   parameter order; padding entries 0) and L (host).  x, t on the device.  Synchronises. */
/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops,
   harnesses that forbid hipMalloc): lbm_nn_forward with the packed input and the hidden
   activations in a fixed scratch array of the library (2.25 MiB per device, held until the
   process ends) instead of the network's workspace.  n h w <= LBM_NN_NOALLOC_MAX_PIXELS
   (LBM_EINVAL beyond), independent of the network's pixel capacity; the same kernels and the
   same arithmetic, so y equals lbm_nn_forward's bitwise.  The device current on the calling
   thread must be the network's.  Allocates nothing.  Every call on a device shares that
   device's scratch and the last call's contents stay there: calls that overlap on one device
   (several streams or threads) race.  Asynchronous on the network's stream. */
#define LBM_NN_NOALLOC_MAX_PIXELS 16384
int lbm_nn_forward_noalloc(lbm_nn* nn, const float* x, float* y, int n, int h, int w);
int lbm_nn_gradient(lbm_nn* nn, const float* x, const float* t, int n, int h, int w, float* grad, double* loss);
/* One Adam step of learning rate lr on L; *loss (optional, synchronises) gets L before the step. */
int lbm_nn_train_step(lbm_nn* nn, const float* x, const float* t, int n, int h, int w, float lr, double* loss);
int lbm_nn_destroy(lbm_nn* nn);
const char* lbm_nn_last_error(const lbm_nn* nn);

/* Coarse input maps of the handle's current state (device FP32, (ny/f) x (nx/f) x 3), the
   coarse target from its current potential ((ny/f) x (nx/f)), and the seeding of its
   current potential links and phi from a coarse deviation map (bilinear between cell
   centres, periodic in x, clamped in y, taken at the centre of each pair of nodes (2k, 2k+1)
   of a row so that both get the same value; links at their equilibria w_i phi).  The pairing
   keeps the seed free of the sweeps' undamped alternating mode: the checkerboard sum of the
   moving links, sum (-1)^(i+j) (l1 + l2 + l3 + l4), changes sign every sweep and never decays,
   and a nonzero one would hold the relative change above the stopping rule for good.
   Asynchronous on the handle's stream. */
int lbm_nn_features(lbm_handle* h, int factor, float* x);
int lbm_nn_target(lbm_handle* h, int factor, float* t);
int lbm_nn_seed(lbm_handle* h, int factor, const float* y);
/* features -> network -> seed, on the handle's stream, using the network's own buffers
   ((nx/f)(ny/f) <= its pixel capacity).  Follow with lbm_solve_potential (or lbm_step). */
int lbm_warm_start(lbm_handle* h, lbm_nn* nn, int factor);
/* From now on every lbm_step seeds its potential solve from the network (maps of the new
   psi and of f_s^n) instead of starting from the previous step's potential; nn = NULL
   restores the plain method.  The network handle must outlive its use here. */
int lbm_set_warm_start(lbm_handle* h, lbm_nn* nn, int factor);
/* Training sample of case c of a batch: its input maps and target (device FP32).  Synchronises. */
int lbm_batch_nn_sample(lbm_batch* b, int c, int factor, float* x, float* t);
/* lbm_warm_start for every case of a batch, one after the other on the batch's stream: case c
   uses the common divisor f_c of nx_c and ny_c that gives ny_c / f_c nearest coarse_rows coarse
   rows (ties: the larger f_c); the network's pixel capacity must hold the largest coarse map
   (LBM_EINVAL otherwise).  Follow with lbm_batch_solve_potential. */
int lbm_batch_warm_start(lbm_batch* b, lbm_nn* nn, int coarse_rows);
/* The potential solve of every case to its own stopping rule (poisson_tol, poisson_max_sweeps;
   Sec. 3.4, R17), 1/tau_l first refreshed from the current psi and f_s, the loops in lockstep
   launches as in lbm_batch_step; each case's count is appended to its sweep log and
   *max_sweeps_done (may be NULL) gets the largest.  Synchronises. */
int lbm_batch_solve_potential(lbm_batch* b, int* max_sweeps_done);

#ifdef __cplusplus
}
#endif
#endif
