// Pointwise, transport and Krylov-vector kernels (launchers).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft.hpp"

namespace tumor {

constexpr int kRedThreads = 256;
constexpr int kRedBlocksMax = 1024;
constexpr int kPartialsPerBlock = 16;
// The partials buffer: kRedBlocksMax blocks of kPartialsPerBlock for the
// reductions, or up to kPartialsCount / kDotStride blocks of an FFT pass with
// one inner-product partial per batched system.
constexpr int kDotStride = 4;
constexpr int kPartialsCount = 65536;
static_assert(kPartialsCount >= kRedBlocksMax * kPartialsPerBlock, "partials buffer");
// Independent systems of a batched solve (the CN solves of i, o and l).
constexpr int kMaxSys = 3;

// Device scalars of one PCG solve.  Written by one-block totalling kernels
// (k_fin_*) from the reduction kernels' per-block partials, except pq and
// alpha: every block of the PCG update totals the inner-product partials of
// the pass before it itself, and block 0 stores them.  Read by the following
// kernels and by the host.
struct SolveScalars {
  double bb;      // ||b||^2 (spectral, Parseval-weighted)
  double rr;      // ||r||^2 of the current residual
  double rho;     // <r, M^-1 r>
  double alpha;
  double beta;
  double pq;      // <p, A p>
  int32_t it;     // iterations taken
  int32_t done;   // 1: no further iteration (converged, limit, breakdown)
  int32_t conv;   // 1: converged
  int32_t bad;    // 1: non-finite or non-positive curvature encountered
  int32_t pad[4];
};

// Voxel means of the coefficient fields and species masses.
struct CoefScalars {
  double Kbar, mubar, lambar, etabar;
  double mass[8];
  int32_t bad;
  int32_t pad[3];
  // Written by the transport (reset before it): bits of non-negative doubles,
  // which order like unsigned integers, so blocks combine them by atomic max.
  unsigned long long cfl_bits;      // max |dt v| / h
  unsigned long long qmax_bits[6];  // max |q| of p, i, n, g, w, f (mixed precision only)
};

// Constants of the coefficient refresh (Eqs. e:diffusion_tensor,
// e:reaction_op, e:lame, e:screening), computed on the host from tumor_params.
struct RefreshConsts {
  double k_w, k_g, k_f;
  double rho_w, rho_g;
  double mu_w, mu_g, mu_f, mu_t;
  double la_w, la_g, la_f, la_t;
  double eta_t, eta_h;
  double mu_b, la_b, eta_b;  // background material
};

struct ReactConsts {
  double dt;
  double alpha0, beta0, gamma, sigma_b, o_hyp, o_inv, o_mit, o_heal;
  double delta_s, delta_p, delta_e, delta_half, delta_l, eps, rho_inv_frac;
  int edema;
};

// Reaction + oxygen + edema + refresh (one pass over the grid).
struct ReactArgs {
  // inputs (after transport and diffusion)
  const double *p, *i_dag, *i_dd, *n, *g, *w, *o, *l, *f;
  // outputs (may alias p, n, g, w, o, l of the inputs; not i_dag)
  double *po, *io, *no, *go, *wo, *oo, *lo, *fo;
  // coefficient fields: rho is read (frozen growth rate) then overwritten
  double *K, *rho, *mu, *lam, *eta;
  float *K32, *mu32, *lam32, *eta32;  // nullable (mixed precision copies)
  const double* bg;                   // static background fraction
  CoefScalars* cs;
  double* partials;
  long long V;
  int do_reaction;
  int single;  // single-species model: tumour c in p (i_dag = c after transport, i_dd after diffusion)
  ReactConsts rc;
  RefreshConsts fc;
};

void launch_react(const ReactArgs& a, hipStream_t st);

// p0 = sum_k w_k exp(-|x - c_k|_per^2 / (2 s_k^2)); ic = n_ic x (cx, cy, cz, s, w)
void launch_ic(int n, const double* ic, int n_ic, double* p0, hipStream_t st);
// p[0 .. count) = value
void launch_fill(double* p, double value, long long count, hipStream_t st);
// dst[0 .. bytes) = src[0 .. bytes); bytes a multiple of 16, both 16-byte aligned
void launch_stream_copy(const void* src, void* dst, long long bytes, hipStream_t st);

// Semi-Lagrangian step (Sec. 3).  v: velocity components and divergence
// (physical).  RC: arithmetic type of the interpolation weights and sums.
struct SLArgs {
  const double *vx, *vy, *vz, *div;
  const double *p, *i, *n, *g, *w, *f;
  double *po, *io, *no, *go, *wo, *fo;
  int n_grid;
  double dt, s;  // s = dt / h
};
// The semi-Lagrangian step (RK2 characteristics, tricubic values from LDS halo
// tiles, Heun source) in the interpolation type RC.  cs->cfl_bits and
// cs->qmax_bits must be zero on entry; max |dt v| / h is max-combined into
// cfl_bits.
template <typename RC>
void launch_sl_tile(const SLArgs& a, CoefScalars* cs, hipStream_t st);

// Tricubic Lagrange interpolation at arbitrary grid-index points.
void launch_interp(int n, const double* q, const double* jx, const double* jy, const double* jz,
                   long long count, double* out, hipStream_t st);

// ---- Krylov vectors in spectral space (ncomp blocks of S = N^3/2 complex)
enum PrecKind : int { PREC_DIFF = 0, PREC_ELAST = 1 };

struct PrecConsts {
  double h;  // dt/2 for CN
  int kind;  // PrecKind
};

struct KrylovArgs {
  void *x, *r, *p, *q, *b;       // complex R arrays (b, ax: see each kernel)
  const void* ax;
  const CoefScalars* cs;
  SolveScalars* sv;
  double* partials;
  int n, ncomp;
  PrecConsts pc;
  double thr2;   // convergence threshold on ||r||^2
  int limit;     // iteration limit (max_it or a forced count)
  int fixed;     // 1: ignore convergence, stop at `limit`
  double scale32;  // launch_residual: r32 = float(scale32 * r), a power of two
  // launch_pcg_update: the inner-product pass's block partials of <p, q>
  // (dnb blocks, dstride apart); every block of the update totals them
  // itself (same order as a one-block kernel) to get alpha = rho / <p, q>
  const double* dpart;
  int dnb, dstride;
};

// r = b - ax (ax nullable: r = b); bb, rr -> sv.  Optionally r32 = float(r).
template <typename R>
void launch_residual(const KrylovArgs& a, void* r32, hipStream_t st);
// CN start from c (= x0) and D c: b = c + h Dc, r = b - (c - h Dc); bb, rr -> sv.
template <typename R>
void launch_cn_residual(const KrylovArgs& a, const void* c, const void* dc, hipStream_t st);
// p = M^-1 r; rho = <r, M^-1 r>; it = 0; done = 0.  zero_x: x = 0 as well.
template <typename R>
void launch_pcg_start(const KrylovArgs& a, int zero_x, hipStream_t st);
// alpha = rho / <p, q> (from the partials at a.dpart), r -= alpha q,
// convergence test, beta.  x += alpha p is deferred: the fused
// p-update pass of the next iteration applies it before replacing p
// (ZPUpdateArgs.x), and launch_pcg_xfinal after the last iteration.
template <typename R>
void launch_pcg_update(const KrylovArgs& a, hipStream_t st);
// x += alpha p for the last iteration that ran (none: no-op)
template <typename R>
void launch_pcg_xfinal(const KrylovArgs& a, hipStream_t st);
// out = M^-1 in (one application of the preconditioner)
template <typename R>
void launch_precond(const KrylovArgs& a, const void* in, void* out, hipStream_t st);
// ---- ns independent systems sharing one operator (the CN solves of i, o, l).
// Vectors hold ns blocks of S complex values; system k has its own scalars
// sv[k] and stopping rule (thr2, limit, fixed).  Only systems whose bit is set
// in `active` are read or written; the finishing kernels mark the others done.
// Each system's arithmetic (and the order of its sums) is that of the
// one-system kernels above.
struct BatchArgs {
  void *x, *r, *p, *q, *b;
  const void* ax;  // nullable (residual: r = b - ax)
  const CoefScalars* cs;
  SolveScalars* sv;  // ns entries
  double* partials;
  int n, ns, active;
  PrecConsts pc;  // PREC_DIFF
  double thr2[kMaxSys];
  int limit[kMaxSys];
  int fixed[kMaxSys];
  double scale32[kMaxSys];  // launch_bresidual: r32 = float(scale32 * r)
  // launch_bpcg_update: system k's <p, q> partials at dpart[block * kDotStride + k], dnb blocks
  const double* dpart;
  int dnb;
};
template <typename R>
void launch_bresidual(const BatchArgs& a, void* r32, hipStream_t st);
template <typename R>
void launch_bcn_residual(const BatchArgs& a, const void* c, const void* dc, hipStream_t st);
template <typename R>
void launch_bpcg_start(const BatchArgs& a, int zero_x, hipStream_t st);
template <typename R>
void launch_bpcg_update(const BatchArgs& a, hipStream_t st);
template <typename R>
void launch_bpcg_xfinal(const BatchArgs& a, hipStream_t st);
// flags[k] = 0 for the systems in mask, 1 for the others (k < ns)
void launch_set_flags(int* flags, int ns, int mask, hipStream_t st);
// x64[k] += s[k] * double(x32[k]) for the systems in mask (blocks of count values)
void launch_badd32to64(void* x64, const void* x32, const double (&s)[kMaxSys], int ns, int mask, long long count,
                       hipStream_t st);

// Mass-effect diagnostics of a displacement (Sec. 3, e:hook, e:princ_stress,
// e:jacobian; Sec. 4 grid search).  f[3a + b'] are physical fields: f[0..2]
// = u_a, then F_ab = G_b u_a stored at f[3 + 3b + a] (derivative b of u_a).
struct DiagArgs {
  const double* f[12];
  const double *mu, *lam;
  const double* ic;  // n_ic x (cx, cy, cz, sigma, weight), device
  int n_ic;
  int n;
  double h;
  double thr;        // displacement threshold, voxels
  double *trace, *shear, *jac;  // nullable outputs
  double* partials;
};
// results[8] = max |u|/h, min tr T, max tr T, max tau, min J, max J,
// sqrt(h^3 sum (J-1)^2), d_max (voxels; 0 without seeds or displacement)
void launch_diag(const DiagArgs& a, double* results, hipStream_t st);


// x64 += s * double(x32)
void launch_add32to64(void* x64, const void* x32, double s, long long count, hipStream_t st);
// physical float -> double
void launch_f32_to_f64(const float* in, double* out, long long count, hipStream_t st);
void launch_scale64(double* x, double s, long long count, hipStream_t st);

}  // namespace tumor
