/*
 * tumor.h -- C ABI of libtumor, an MI355X (gfx950) implementation of one
 * operator-split time step of the multispecies glioblastoma model with mass
 * effect of Subramanian, Gholami & Biros (arXiv 1810.05370).
 *
 * Model and discretisation this library implements:
 *   - species p, i, n (proliferative, invasive, necrotic tumour cells), o
 *     (oxygen), l (edema), g, w (gray, white matter), f (CSF) on the periodic
 *     cube [0, 2*pi)^3 with N^3 nodes (Sec. 3, fictitious domain);
 *   - the PDE system of Eq. e:gog (Sec. 2.3) with the edema equation e:edema
 *     (Sec. 2.4) and the screened elasticity e:screening with Lame fields
 *     e:lame (Sec. 2.1);
 *   - the multispecies splitting of Sec. 3: semi-Lagrangian transport,
 *     Crank-Nicolson diffusion by preconditioned CG, explicit reaction,
 *     oxygen and edema updates, coefficient refresh, and the elasticity
 *     solve by PCG with the constant-Lame spectral preconditioner.
 *
 * Conventions for every entry point:
 *   - Real arrays are FP64, N^3 elements, C order [z][y][x] (x fastest).
 *     Vector fields are three such blocks (x, y, z components) back to back.
 *   - Array arguments are DEVICE pointers unless marked "host".  The caller
 *     owns every pointer it passes; inputs are copied, never retained, except
 *     the workspace, which must stay valid until tumor_destroy.
 *   - All work is queued on the HIP stream given to tumor_init.  Each call
 *     returns after its work has completed (PCG control reads scalars back).
 *   - Every call returns a tumor_status.  No C++ exception crosses the ABI.
 *     On a non-OK status, tumor_last_error() returns a message (thread-local).
 *   - Arguments are validated before any device work: a bad pointer/size/enum
 *     gives TUMOR_EINVAL and leaves the context unchanged.
 *   - A context is single-threaded: calls on one context must not overlap.
 *   - Device memory is never allocated after tumor_init; tumor_init itself
 *     only carves the caller's workspace (it allocates a few hundred bytes of
 *     pinned host memory for scalar read-back).
 */
#ifndef TUMOR_H
#define TUMOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TUMOR_ABI_VERSION 3

typedef enum {
  TUMOR_OK = 0,
  TUMOR_EINVAL = -1,   /* invalid argument (checked before any device work)     */
  TUMOR_ENOMEM = -2,   /* workspace smaller than tumor_workspace_bytes reports  */
  TUMOR_ENOCONV = -3,  /* a PCG solve hit max_it; state holds the last iterate  */
  TUMOR_EDEVICE = -4,  /* HIP runtime error (no device, launch failure, ...)    */
  TUMOR_ENAN = -5,     /* a residual norm became NaN/Inf                        */
  TUMOR_ESTATE = -6    /* call out of order (e.g. adjoint without a record)     */
} tumor_status;

typedef enum {
  TUMOR_PREC_FP64 = 0,  /* every kernel in FP64                                  */
  TUMOR_PREC_MIXED = 1  /* FP32 FFTs, operator applies and interpolation; FP64
                           species, reaction thresholds, PCG dot products and an
                           outer FP64 residual correction of every solve         */
} tumor_precision;

/* Sub-step switches (tumor_config.flags). */
#define TUMOR_F_ADVECTION  0x1  /* semi-Lagrangian transport (Sec. 3)          */
#define TUMOR_F_ELASTICITY 0x2  /* mass-effect elasticity solve (Sec. 3)       */
#define TUMOR_F_EDEMA      0x4  /* edema diffusion + reaction (Sec. 2.4)        */
#define TUMOR_F_DEFAULT    (TUMOR_F_ADVECTION | TUMOR_F_ELASTICITY | TUMOR_F_EDEMA)
#define TUMOR_F_ADJOINT    0x8  /* reserve adjoint scratch in the workspace      */
/* Symmetric (Strang) form of the step (Sec. 3 names Strang splitting; the
 * default is the listed sequential order).  With TUMOR_F_ADVECTION set, each
 * step transports over dt/2, refreshes the coefficients from that state (its
 * K, rho and means drive the diffusion and reaction), runs diffusion and
 * reaction over dt, transports over dt/2 again with the same velocity, then
 * refreshes and solves the elasticity.  Oxygen and edema are not transported
 * in either form.  Without TUMOR_F_ADVECTION the flag changes nothing.
 * Forward only: rejected together with TUMOR_F_ADJOINT. */
#define TUMOR_F_STRANG     0x10

/* Model parameters.  Names follow Table t:setup (Sec. 2.5) and the equations
 * they enter:
 *   K      = k_w w + k_g g + k_f f                       (e:diffusion_tensor)
 *   rho_p  = rho_w w + rho_g g,  rho_i = rho_inv_frac * rho_p
 *                                                  (e:reaction_op, e:gog_reac_inv_op)
 *   alpha  = alpha0 H(o_inv - o), beta = beta0 H(sigma_b - p - i) o,
 *   h      = gamma H(o_hyp - o), o_mit = (o_hyp + o_inv)/2
 *                                  (e:alpha, e:beta, e:death, e:gog_reac_op)
 *   oxygen: -delta_p p + delta_s (o_heal - o)(g + w)                    (e:ox)
 *   edema:  delta_e i/(i + delta_half)(1 - i) - delta_l l             (e:edema)
 *   eta    = eta_tumor (p+i+n) + eta_healthy (g+w+f) + eta_bg bg  (e:screening)
 *            (all >= 0, not all zero: without screening the operator vanishes on
 *            the modes whose derivative symbols are all zero -- the mean and
 *            the Nyquist corner modes -- and the system has no solution)
 *   mu, lambda from (E_s, nu_s) of w, g, f, the tumour p+i+n and the
 *           background bg (e:lame), both multiplied by lame_scale
 *   force  b = zeta tanh(p+n) grad(p+n)                   (e:forcingfunction)
 *   H(x)   = (1 + tanh(x / heaviside_eps)) / 2  (the smoothed Heaviside)
 */
typedef struct {
  double k_w, k_g, k_f;
  double rho_w, rho_g, rho_inv_frac;
  double alpha0, beta0, gamma, sigma_b, o_hyp, o_inv, o_heal, delta_s, delta_p;
  double delta_e, delta_half, delta_l;
  double eta_tumor, eta_healthy;
  double E_wm, E_gm, E_csf, E_tumor, nu_wm, nu_gm, nu_csf, nu_tumor;
  double lame_scale, zeta;
  double heaviside_eps;
  double E_bg, nu_bg, eta_bg;  /* background material (fictitious domain, Sec. 3;
                                  Table t:setup): with the background fraction
                                  TUMOR_FIELD_BG it adds to the Lame mixture and
                                  the screening, penalising displacement outside
                                  the brain; it has no diffusion or growth, so
                                  the tumour flux vanishes there               */
} tumor_params;

/* Tumour model (tumor_config.model).
 *   MULTISPECIES: p, i, n, o, l, g, w, f (Sec. 2.3-2.4, Eq. e:gog, e:edema).
 *   SINGLE: the reaction-diffusion model with mass effect (Sec. 2.2, Eq. e:rd):
 *     one tumour density c (stored in the p field; i, n, l stay 0 and o stays
 *     o_heal) that diffuses with K and grows as rho c (1 - c), rho = rho_w w +
 *     rho_g g (e:reac_op, e:reaction_op); g and w lose the tumour's diffusion
 *     and growth increments in proportion g : w (e:gm, e:wm); the force is
 *     zeta tanh(c) grad c (e:force).  Split as in the single-species list of
 *     Sec. 3: transport, CN diffusion of c, reaction, refresh, elasticity.
 *     Parameters of the multispecies reaction (alpha0, ..., delta_l) are
 *     unused; TUMOR_F_EDEMA has no effect and TUMOR_F_ADJOINT is rejected. */
typedef enum { TUMOR_MODEL_MULTISPECIES = 0, TUMOR_MODEL_SINGLE = 1 } tumor_model;

/* Numerical configuration (Table t:numparams: N, dt, Krylov tolerance). */
typedef struct {
  int32_t n;            /* grid size per axis: a power of two in [16, 512]     */
  int32_t precision;    /* tumor_precision                                       */
  double dt;            /* time step (> 0)                                       */
  double rtol_diff;     /* CN diffusion PCG relative tolerance, in (0, 1)        */
  double rtol_elast;    /* elasticity PCG relative tolerance, in (0, 1)          */
  int32_t max_it;       /* PCG iteration cap per solve (>= 1)                    */
  int32_t flags;        /* TUMOR_F_* (0 selects TUMOR_F_DEFAULT)                 */
  int32_t model;        /* tumor_model                                           */
  int32_t reserved[3];  /* must be zero                                          */
} tumor_config;

/* Statistics of the last step (or solve). */
typedef struct {
  int32_t it_diff[3];        /* CG iterations: invasive cells, oxygen, edema   */
  int32_t it_elast;          /* elasticity PCG iterations (inner, summed)      */
  int32_t outer_elast;       /* FP64 outer corrections (mixed precision)       */
  int32_t outer_diff[3];     /* FP64 outer corrections of the three CN solves  */
  double relres_diff[3];     /* final relative residuals (FP64)                */
  double relres_elast;
  double mass[8];            /* h^3 sum of p, i, n, o, l, g, w, f               */
  double max_cfl;            /* max |dt v| / h of the velocity that was used
                                (full dt also for TUMOR_F_STRANG)               */
} tumor_step_stats;

typedef struct tumor_ctx tumor_ctx;

/* Field identifiers for tumor_get_field / tumor_set_field. */
enum {
  TUMOR_FIELD_P = 0, TUMOR_FIELD_I, TUMOR_FIELD_N, TUMOR_FIELD_O, TUMOR_FIELD_L,
  TUMOR_FIELD_G, TUMOR_FIELD_W, TUMOR_FIELD_F,
  TUMOR_FIELD_U = 8,        /* displacement u^n, 3 N^3 values                 */
  TUMOR_FIELD_UPREV = 9,    /* displacement u^{n-1}, 3 N^3 values             */
  TUMOR_FIELD_K = 10, TUMOR_FIELD_RHO = 11, TUMOR_FIELD_MU = 12,
  TUMOR_FIELD_LAMBDA = 13, TUMOR_FIELD_ETA = 14,   /* coefficients, read only */
  TUMOR_FIELD_BG = 15,      /* static background-material fraction (0 at init;
                               call tumor_refresh after setting it)            */
  TUMOR_FIELD_COUNT = 16
};

/* Device workspace size (bytes) a context for `cfg` needs.  Host arguments.
 * Returns TUMOR_EINVAL for an invalid configuration. */
int tumor_workspace_bytes(const tumor_config* cfg, size_t* bytes);

/* Create a context and its initial state (Sec. 3 initial conditions, Eq. e:gog):
 *   g0, w0, f0 <- gm, wm, csf (device, copied);
 *   p0 = sum_k ic_weights[k] exp(-d(x, c_k)^2 / (2 ic_sigmas[k]^2)), d the
 *        periodic minimum-image distance, c_k = ic_centers[3k..3k+2] as (x,y,z);
 *   i0 = n0 = l0 = 0, o0 = o_heal, u^0 = u^-1 = 0; coefficients from q0.
 * ic_centers, ic_sigmas, ic_weights are HOST arrays of n_ic >= 0 entries.
 * workspace: device buffer of ws_bytes >= tumor_workspace_bytes(cfg), 256-byte
 * aligned, owned by the caller, used exclusively by this context.
 * hip_stream: a hipStream_t (NULL = the null stream). */
int tumor_init(tumor_ctx** out, const tumor_config* cfg, const tumor_params* prm,
               void* workspace, size_t ws_bytes,
               const double* wm, const double* gm, const double* csf,
               int32_t n_ic, const double* ic_centers, const double* ic_sigmas,
               const double* ic_weights, void* hip_stream);

/* Allocation-free context, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same as tumor_init, with the same arguments except the
 * workspace: the context carves a fixed array of TUMOR_STATIC_WS_BYTES that the
 * library itself holds on each GPU it runs on (reserved with the code object,
 * kept until the process ends), and its host storage (scalar read-back, the
 * initial-condition table) is static too.  The call allocates no device or
 * pinned host memory and calls no allocating routine on success (an error
 * message is a host string).
 *   Limits: tumor_workspace_bytes(cfg) <= TUMOR_STATIC_WS_BYTES (every n <= 32,
 *   both precisions, with or without TUMOR_F_ADJOINT), n_ic <= 256; otherwise
 *   TUMOR_EINVAL with a message, before any device work.
 *   One such context per GPU at a time: while one is live on the current device
 *   a second call returns TUMOR_ESTATE.  tumor_destroy releases the array.  The
 *   array keeps the last context's contents; tumor_init_static clears whatever
 *   must start at zero.  Contexts of the same GPU created on different threads
 *   would race on the array, which is why a second live one is refused.
 *   Every other entry point works on such a context as on any other; a tape
 *   for the adjoint (tumor_record) is still caller memory. */
#define TUMOR_STATIC_WS_BYTES (32u << 20)
int tumor_init_static(tumor_ctx** out, const tumor_config* cfg, const tumor_params* prm,
                      const double* wm, const double* gm, const double* csf,
                      int32_t n_ic, const double* ic_centers, const double* ic_sigmas,
                      const double* ic_weights, void* hip_stream);

/* Advance nsteps split steps (Sec. 3, multispecies splitting).  `last` (host,
 * nullable) receives the statistics of the final step.  TUMOR_ENOCONV: a solve
 * hit max_it (the step still completed with the last iterate). */
int tumor_step(tumor_ctx* ctx, int32_t nsteps, tumor_step_stats* last);

/* Solve the screened elasticity system (eta - L) u = -b (the SPD form of
 * Eq. e:screening) with the context's current coefficients, starting from the
 * current displacement u^n.  force: 3 N^3 device array b, or NULL to use
 * b = zeta tanh(p+n) grad(p+n) of the current state.  u_out: 3 N^3 device
 * output.  iters / relres: host outputs (nullable).  The state is unchanged. */
int tumor_solve_elasticity(tumor_ctx* ctx, const double* force, double* u_out,
                           int32_t* iters, double* relres);

/* Run the transport sub-step alone on the current state (Sec. 3, first two
 * items of the multispecies splitting): velocity u_t^n = (u^n - u^{n-1}) / dt
 * and the semi-Lagrangian step of p, i, n, g, w (conservative form) and f,
 * exactly as tumor_step does it.  out: device, 6 N^3 values, the transported
 * p, i, n, g, w, f in that order.  max_cfl: host, nullable, receives
 * max |dt u_t^n| / h.  The step is always the full-dt one, also for a context
 * created with TUMOR_F_STRANG.  The state is unchanged. */
int tumor_transport(tumor_ctx* ctx, double* out, double* max_cfl);

/* Mass-effect diagnostics of the current displacement u^n (Sec. 3: stress by
 * Hooke's law e:hook, principal stresses shown by the stress trace, maximum
 * shear from Mohr's circle e:princ_stress, Jacobian e:jacobian; Sec. 4: the
 * grid-search scalars).  With F_ab = G_b u_a (spectral derivatives) and the
 * context's current Lame fields:
 *   trace     = tr T,  T = lambda tr(F) I + mu (F + F^T)
 *   shear     = sqrt(((T_xx - T_yy)/2)^2 + T_xy^2)   (x-y plane, as printed)
 *   J         = det(I + F)
 * fields: device, 3 N^3 values (trace, shear, J), or NULL for the scalars
 * only.  threshold: displacement (voxels) whose contour defines d_max.
 * Runs in FP64 in both precisions; the state is unchanged. */
typedef struct {
  double max_disp;             /* max |u| / h (voxels)                            */
  double trace_min, trace_max; /* extremes of the stress trace                    */
  double shear_max;            /* max of the Mohr shear stress                    */
  double jac_min, jac_max;     /* extremes of J                                   */
  double jac_l2;               /* sqrt(h^3 sum (J - 1)^2)                         */
  double d_max;                /* max distance (voxels, periodic) from the nearest
                                  initial seed of the points with |u| >= threshold
                                  voxels; 0 without seeds or such points          */
} tumor_diagnostics;
int tumor_diagnose(tumor_ctx* ctx, double threshold, double* fields, tumor_diagnostics* out);

/* Discrete adjoint (the exact transpose of the linearised split step, every
 * PCG solve taken as exact; the paper leaves adjoint-based inversion to
 * future work, Sec. 5).  Requires a context created with TUMOR_F_ADJOINT.
 *
 * tumor_record(ctx, nsteps, ckpt_every, tape, tape_bytes): the next nsteps
 * calls of tumor_step are recorded into `tape` (device, 256-byte aligned,
 * >= tumor_tape_bytes(cfg, nsteps, ckpt_every)).
 *   ckpt_every = 1: every state and, per step, the 8 intermediate fields the
 *     transposes read are kept ((nsteps + 1) * 14 + nsteps * 8 fields of N^3
 *     doubles); the reverse sweep recomputes no forward step.
 *   ckpt_every = K > 1: the full state (species and both displacements) is
 *     checkpointed every K steps; the tape also holds a window of K states
 *     that the reverse sweep recomputes from the nearest checkpoint, plus one
 *     recomputed forward step per reversed step (about 14 (nsteps / K + K)
 *     fields). 
 *
 * tumor_adjoint_step(ctx, adj, grad): reverses the latest recorded step not
 * yet reversed.  adj: device, 14 N^3 values, the adjoint of the state
 * (p, i, n, o, l, g, w, f, u_x, u_y, u_z, uprev_x, uprev_y, uprev_z) after
 * that step on input, before it on output.  grad: host, 5 + n_ic doubles,
 * accumulated: d/d(rho, k_w, k_g, k_f, lame_scale, ic_weights[0..n_ic)),
 * where rho moves rho_w and rho_g together; the ic_weights part is added when
 * the first step (step 0) is reversed.  The forward state of the context is
 * overwritten by the recomputation (it holds the state after the reversed
 * step on return).  TUMOR_ESTATE: no recording, or every step reversed. */
int tumor_tape_bytes(const tumor_config* cfg, int32_t nsteps, int32_t ckpt_every, size_t* bytes);
int tumor_record(tumor_ctx* ctx, int32_t nsteps, int32_t ckpt_every, void* tape, size_t tape_bytes);
int tumor_adjoint_step(tumor_ctx* ctx, double* adj, double* grad);

/* State snapshots (checkpoint and restore of the time-stepping state of
 * Sec. 3: the species p, i, n, o, l, g, w, f and the displacements u^n,
 * u^{n-1} that define the backward-difference velocity).  The snapshot holds
 * the library's internal representation, so a restored context steps exactly
 * as the saved one would have (bit for bit).
 *   tumor_state_bytes: size of one snapshot for cfg (host arguments).
 *   tumor_save_state: copy the current state into dst (device, >= bytes,
 *     8-byte aligned); the snapshot starts with a small header naming n.
 *   tumor_load_state: replace the current state by the snapshot in src
 *     (device, 8-byte aligned) and refresh the coefficients from it.  A
 *     snapshot of another grid size (or not a snapshot) gives TUMOR_EINVAL and
 *     leaves the state unchanged; one of the other precision is accepted (the
 *     state is FP64 in both).  TUMOR_ESTATE while a recording (tumor_record) or
 *     its reverse sweep is unfinished; a finished recording is released.
 *     Buffers are caller-owned. */
int tumor_state_bytes(const tumor_config* cfg, size_t* bytes);
int tumor_save_state(tumor_ctx* ctx, void* dst, size_t bytes);
int tumor_load_state(tumor_ctx* ctx, const void* src, size_t bytes);

/* Copy a field out of / into the state (device arrays of N^3, or 3 N^3 for
 * TUMOR_FIELD_U and TUMOR_FIELD_UPREV).  Coefficient fields are read only;
 * setting a species or the background refreshes nothing (call tumor_refresh
 * afterwards to recompute the coefficients). */
int tumor_get_field(tumor_ctx* ctx, int32_t field_id, double* dst);
int tumor_set_field(tumor_ctx* ctx, int32_t field_id, const double* src);
int tumor_refresh(tumor_ctx* ctx);

/* Building blocks of the step, exposed for verification.  Device arrays.
 *   TUMOR_OP_DERIV_X/Y/Z : out = G_a in (spectral derivative, Nyquist dropped)
 *   TUMOR_OP_DIFFUSION   : out = div(K grad in), K of the current state
 *   TUMOR_OP_ELASTICITY  : out = (eta - L) in on 3 N^3 arrays
 *   TUMOR_OP_ELAST_PRECOND: out = constant-Lame inverse of in (3 N^3)
 *   TUMOR_OP_CN_PRECOND  : out = constant-K CN inverse of in
 *   TUMOR_OP_FORCE       : out (3 N^3) = zeta tanh(in) grad(in)
 * In the mixed mode these run in FP32. */
enum {
  TUMOR_OP_DERIV_X = 0, TUMOR_OP_DERIV_Y = 1, TUMOR_OP_DERIV_Z = 2,
  TUMOR_OP_DIFFUSION = 3, TUMOR_OP_ELASTICITY = 4, TUMOR_OP_ELAST_PRECOND = 5,
  TUMOR_OP_CN_PRECOND = 6, TUMOR_OP_FORCE = 7, TUMOR_OP_COUNT = 8
};
int tumor_apply_op(tumor_ctx* ctx, int32_t op, const double* in, double* out);

/* Semi-Lagrangian interpolation: out[k] = tricubic Lagrange interpolant of
 * the periodic field q at grid-index coordinates (jx[k], jy[k], jz[k]),
 * k < count (device arrays, 0 <= count < 2^40). */
int tumor_interp(tumor_ctx* ctx, const double* q, const double* jx, const double* jy,
                 const double* jz, int64_t count, double* out);

/* Verification hook for the FP64 precision: run the four solves of the next
 * step (invasive-cell, oxygen and edema CN solves, elasticity) for exactly
 * iters[k] PCG iterations each (-1 = stop on the tolerance as usual), so that
 * two implementations can be compared in iteration lockstep.  iters: host
 * array of 4 values, or NULL to clear.  TUMOR_EINVAL in the mixed precision. */
int tumor_force_iterations(tumor_ctx* ctx, const int32_t* iters);

/* Measurement hook: bracket every launch of one kernel class (each class is
 * one kernel symbol, except XOTHER, SL, KRYLOV64/32) with HIP events
 * on the context's stream and accumulate launches, elapsed milliseconds and
 * the algorithmic HBM bytes of those launches (each input and output array
 * counted once).  enable = 1 resets and starts, 0 stops.  Reading flushes
 * pending events (it synchronises the stream). */
enum {
  TUMOR_K_COLINV64 = 0, TUMOR_K_COLFWD64, TUMOR_K_COLINV32, TUMOR_K_COLFWD32, TUMOR_K_XELAST64,
  TUMOR_K_XELAST32, TUMOR_K_XDIFF64, TUMOR_K_XDIFF32, TUMOR_K_XOTHER, TUMOR_K_SL, TUMOR_K_REACT,
  TUMOR_K_KRYLOV64, TUMOR_K_KRYLOV32,
  TUMOR_K_ZINVP64, TUMOR_K_ZINVP32,      /* first pass with the fused direction update
                                            (elasticity, 3 components)                 */
  TUMOR_K_COLDOT64, TUMOR_K_COLDOT32,    /* last pass with the fused inner product      */
  TUMOR_K_COLINV32Z, TUMOR_K_COLFWD32Z,  /* FP32 z passes (COLINV32/COLFWD32: y passes)  */
  TUMOR_K_ZINVP64_1, TUMOR_K_ZINVP32_1,  /* fused first pass of a one-field CN solve      */
  TUMOR_K_ZINVPB64, TUMOR_K_ZINVPB32,    /* fused first pass of the batched CN solve of
                                            i, o and l                                 */
  TUMOR_K_COUNT
};
int tumor_kernel_timer(tumor_ctx* ctx, int32_t kernel_class, int32_t enable);
int tumor_kernel_timer_read(tumor_ctx* ctx, int32_t kernel_class, int64_t* launches, double* ms,
                            double* bytes);

/* Measurement hook: time every step's sub-steps (Sec. 3 splitting) with HIP
 * events on the context's stream.  enable = 1 resets and starts, 0 stops.
 * tumor_substep_timer_read: steps timed and ms (host, TUMOR_SUB_COUNT doubles)
 * summed per sub-step: transport (both halves of the symmetric form, with the
 * velocity), diffusion (the CN solves), reaction (reaction, oxygen, edema and
 * the coefficient refresh), elasticity (force, solve and rotation).  The step
 * also opens a roctx range per sub-step ("tumor transport", ...), which
 * rocprofv3 --marker-trace records whether or not this timer is on. */
enum { TUMOR_SUB_TRANSPORT = 0, TUMOR_SUB_DIFFUSION = 1, TUMOR_SUB_REACTION = 2, TUMOR_SUB_ELASTICITY = 3,
       TUMOR_SUB_COUNT = 4 };
int tumor_substep_timer(tumor_ctx* ctx, int32_t enable);
int tumor_substep_timer_read(tumor_ctx* ctx, int64_t* steps, double* ms);

/* Measurement hook: copy `bytes` (a multiple of 16, below 2^42) from src to
 * dst (device pointers, 16-byte aligned, not overlapping) with a streaming
 * kernel of one 16-byte load and store per thread, queued on hip_stream (NULL =
 * the null stream); returns without waiting.  Its rate (2 bytes moved per byte
 * copied) is the achievable HBM bandwidth that the other kernels' rates are
 * set against.  TUMOR_EINVAL for a bad argument, before any device work. */
int tumor_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream);

void tumor_destroy(tumor_ctx* ctx);
const char* tumor_last_error(void);
int tumor_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TUMOR_H */
