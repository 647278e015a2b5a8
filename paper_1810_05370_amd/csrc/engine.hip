// libtumor host engine: workspace layout, operator sequences, PCG control and
// the C ABI declared in include/tumor.h.
//
// State on the device (FP64): species p, i, n, o, l, g, w, f (physical) and
// the displacements u^n, u^{n-1} in packed spectral form (see passes.hpp).
// Every Krylov solve runs in spectral space: vectors are spectra, the
// preconditioners are diagonal (diffusion) or 3x3 per mode (elasticity), and
// inner products are Parseval-weighted sums, which equal N^3 times the
// physical inner products, so the iterates are those of the physical-space
// method.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "adjoint.hpp"
#include "kernels.hpp"
#include "passes.hpp"
#include "tumor.h"

namespace {

thread_local std::string g_err;

struct Fail : std::runtime_error {
  int code;
  Fail(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHECK(expr)                                                                      \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw Fail(TUMOR_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

using tumor::cplx;
using tumor::ColProg;
using tumor::ColTerm;
using tumor::SYM_IW;
using tumor::SYM_ONE;
using tumor::SYM_RAW;
using tumor::XProg;

template <typename R>
struct PrecBufs {
  cplx<R>* A[8];
  cplx<R>* B[8];
  cplx<R>* x;  // Krylov vectors, 3 blocks of S each
  cplx<R>* r;
  cplx<R>* p;
  cplx<R>* q;
  void* tw;
  const R* K;
  const R* mu;
  const R* lam;
  const R* eta;
};

struct Carver {
  char* base;
  size_t off;
  bool dry;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = dry ? nullptr : reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

bool valid_n(int n) { return n >= 16 && n <= 512 && (n & (n - 1)) == 0; }

int check_cfg(const tumor_config* c) {
  if (!c) return TUMOR_EINVAL;
  if (!valid_n(c->n)) return TUMOR_EINVAL;
  if (c->precision != TUMOR_PREC_FP64 && c->precision != TUMOR_PREC_MIXED) return TUMOR_EINVAL;
  if (!(c->dt > 0.0) || !std::isfinite(c->dt)) return TUMOR_EINVAL;
  if (!(c->rtol_diff > 0.0 && c->rtol_diff < 1.0)) return TUMOR_EINVAL;
  if (!(c->rtol_elast > 0.0 && c->rtol_elast < 1.0)) return TUMOR_EINVAL;
  if (c->max_it < 1) return TUMOR_EINVAL;
  if (c->flags & ~(TUMOR_F_DEFAULT | TUMOR_F_ADJOINT | TUMOR_F_STRANG)) return TUMOR_EINVAL;
  if ((c->flags & TUMOR_F_STRANG) && (c->flags & TUMOR_F_ADJOINT)) return TUMOR_EINVAL;
  if (c->model != TUMOR_MODEL_MULTISPECIES && c->model != TUMOR_MODEL_SINGLE) return TUMOR_EINVAL;
  if (c->model == TUMOR_MODEL_SINGLE && (c->flags & TUMOR_F_ADJOINT)) return TUMOR_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (c->reserved[k] != 0) return TUMOR_EINVAL;
  return TUMOR_OK;
}

constexpr int kMaxPend = 1024;

// Event timing of one kernel class (measurement hook).
struct KTimer {
  int on;
  int pending;
  long long launches;
  double ms;
  double bytes;
  hipEvent_t ev[2 * kMaxPend];
  double pend_bytes[kMaxPend];
  double pend_sys[kMaxPend];  // batched launches: bytes per system still iterating
  int pend_tag[kMaxPend];
};

}  // namespace

struct tumor_ctx {
  tumor_config cfg;
  tumor_params prm;
  hipStream_t st;
  int n;
  long long V, S;
  bool mixed;
  double* BG;   // static background-material fraction
  bool adj;     // adjoint scratch present
  bool single;  // single-species model (tumour c in F[P])
  int flags;
  double* F[8];
  double* G[8];
  double* Rdd[3];  // diffusion outputs i'', o', l' (kept for the adjoint)
  // adjoint scratch (TUMOR_F_ADJOINT)
  double *MB, *LB, *EB, *TB, *T[4], *Y[3], *KB, *RB, *IDD, *DDB, *SLO[6], *DB, *VB[3];
  tumor::GradScalars* gs;
  // recording for the adjoint
  char* tape;
  size_t tape_bytes;
  int rec_active, rec_nsteps, rec_K, rec_steps, rev_done, win_start;
  int n_ic;
  double* ic_host;  // n_ic x (cx, cy, cz, sigma, weight)
  cplx<double>* U;
  cplx<double>* Up;
  cplx<double>* Un;
  double *K, *rho, *mu, *lam, *eta;
  float *K32, *mu32, *lam32, *eta32;
  double* vel[4];
  cplx<double>* b64;
  PrecBufs<double> p64;
  PrecBufs<float> p32;
  tumor::SolveScalars* sv64;  // kMaxSys entries (one per system of a batched solve)
  tumor::SolveScalars* sv32;
  int* bflag;                 // per-system skip flags of the batched FP64 applies
  tumor::CoefScalars* cs;
  double* partials;
  double* dpart;  // inner-product partials of the last pass of a Krylov apply (read by the update)
  // host side
  tumor::SolveScalars* hsv;  // kMaxSys entries
  tumor::CoefScalars* hcs;
  int pred[8];
  int pred_in[8][3];  // mixed precision: inner iterations of outer pass 0, 1, >= 2
  int forced[4];
  bool has_forced;
  tumor::RefreshConsts fc;
  tumor::ReactConsts rc;
  KTimer* timers[TUMOR_K_COUNT];
  int cur_tag;  // PCG iteration index of the launches being queued (-1 outside loops)
  // batched solve in progress (timer accounting): a launch's bytes are split
  // over bsys_total systems, of which bsys_active are computed outside the
  // iterations; within them, a system counts while tag < batch_it[system]
  int bsys_total, bsys_active;
  int batch_ns;
  int batch_it[tumor::kMaxSys];
  int static_dev;  // device of an allocation-free context (tumor_init_static), else -1
  // sub-step timer (tumor_substep_timer): events at the sub-step boundaries of
  // every step, elapsed times summed per sub-step after the step's final sync
  bool sub_on;
  hipEvent_t sub_ev[6];
  double sub_ms[TUMOR_SUB_COUNT];
  long long sub_steps;
};

namespace {

using Ctx = tumor_ctx;

void timer_flush(Ctx& c, int cls, int valid_tag) {
  KTimer* t = c.timers[cls];
  if (!t || t->pending == 0) return;
  HIPCHECK(hipEventSynchronize(t->ev[2 * t->pending - 1]));
  for (int k = 0; k < t->pending; ++k) {
    double bytes = t->pend_bytes[k];
    if (t->pend_sys[k] > 0.0) {
      // a batched launch within the iterations: the systems still iterating did work
      int nact = 0;
      for (int q = 0; q < c.batch_ns; ++q) nact += t->pend_tag[k] < c.batch_it[q] ? 1 : 0;
      if (nact == 0) continue;
      bytes += t->pend_sys[k] * nact;
    } else if (t->pend_tag[k] >= valid_tag) {
      continue;  // launch skipped on the device (solve already done)
    }
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, t->ev[2 * k], t->ev[2 * k + 1]));
    t->ms += ms;
    t->bytes += bytes;
    t->launches += 1;
  }
  t->pending = 0;
}

void timers_flush(Ctx& c, int valid_tag) {
  for (int k = 0; k < TUMOR_K_COUNT; ++k) timer_flush(c, k, valid_tag);
}

// Launch f(), bracketed by events if the class is being timed.  `fixed`
// bytes, plus `per_sys` bytes for each system of a batched solve that the
// launch computes.
template <typename F>
void timed_b(Ctx& c, int cls, double fixed, double per_sys, F&& f) {
  KTimer* t = c.timers[cls];
  if (!t || !t->on) {
    f();
    return;
  }
  if (t->pending == kMaxPend) timer_flush(c, cls, c.cur_tag < 0 ? 0x7fffffff : c.cur_tag);
  HIPCHECK(hipEventRecord(t->ev[2 * t->pending], c.st));
  f();
  HIPCHECK(hipEventRecord(t->ev[2 * t->pending + 1], c.st));
  if (c.cur_tag < 0) {
    // outside the iterations the host knows which systems are computed
    t->pend_bytes[t->pending] = fixed + per_sys * c.bsys_active;
    t->pend_sys[t->pending] = 0.0;
  } else {
    t->pend_bytes[t->pending] = fixed;
    t->pend_sys[t->pending] = per_sys;
  }
  t->pend_tag[t->pending] = c.cur_tag < 0 ? -1 : c.cur_tag;
  t->pending++;
}

// Launch f() timed with `bytes`; within a batched apply (bsys_total > 0) the
// bytes are those of all its systems, split evenly.
template <typename F>
void timed(Ctx& c, int cls, double bytes, F&& f) {
  if (c.bsys_total > 0) timed_b(c, cls, 0.0, bytes / c.bsys_total, f);
  else timed_b(c, cls, bytes, 0.0, f);
}

template <typename R>
constexpr int kcls(int k64, int k32) {
  return sizeof(R) == 8 ? k64 : k32;
}

void layout(Ctx& c, Carver& cv) {
  const long long V = c.V, S = c.S;
  for (int k = 0; k < 8; ++k) c.F[k] = cv.take<double>(V);
  for (int k = 0; k < 8; ++k) c.G[k] = cv.take<double>(V);
  c.U = cv.take<cplx<double>>(3 * S);
  c.Up = cv.take<cplx<double>>(3 * S);
  c.Un = cv.take<cplx<double>>(3 * S);
  c.BG = cv.take<double>(V);
  c.K = cv.take<double>(V);
  c.rho = cv.take<double>(V);
  c.mu = cv.take<double>(V);
  c.lam = cv.take<double>(V);
  c.eta = cv.take<double>(V);
  for (int k = 0; k < 4; ++k) c.vel[k] = cv.take<double>(V);
  c.b64 = cv.take<cplx<double>>(3 * S);
  // The 16 FP64 pass buffers are one contiguous block.
  cplx<double>* ab = cv.take<cplx<double>>(16 * S);
  for (int k = 0; k < 8; ++k) c.p64.A[k] = ab + k * S;
  for (int k = 0; k < 8; ++k) c.p64.B[k] = ab + (8 + k) * S;
  c.p64.x = nullptr;  // the elasticity solve iterates directly in Un
  c.p64.r = cv.take<cplx<double>>(3 * S);
  c.p64.p = cv.take<cplx<double>>(3 * S);
  c.p64.q = cv.take<cplx<double>>(3 * S);
  c.p64.tw = cv.take<cplx<double>>(c.n);
  c.p64.K = c.K;
  c.p64.mu = c.mu;
  c.p64.lam = c.lam;
  c.p64.eta = c.eta;
  c.K32 = c.mu32 = c.lam32 = c.eta32 = nullptr;
  if (c.mixed) {
    c.K32 = cv.take<float>(V);
    c.mu32 = cv.take<float>(V);
    c.lam32 = cv.take<float>(V);
    c.eta32 = cv.take<float>(V);
    for (int k = 0; k < 8; ++k) c.p32.A[k] = cv.take<cplx<float>>(S);
    for (int k = 0; k < 8; ++k) c.p32.B[k] = cv.take<cplx<float>>(S);
    c.p32.x = cv.take<cplx<float>>(3 * S);
    c.p32.r = cv.take<cplx<float>>(3 * S);
    c.p32.p = cv.take<cplx<float>>(3 * S);
    c.p32.q = cv.take<cplx<float>>(3 * S);
  } else {
    std::memset(&c.p32, 0, sizeof(c.p32));
  }
  c.p32.tw = cv.take<cplx<float>>(c.n);
  c.p32.K = c.K32;
  c.p32.mu = c.mu32;
  c.p32.lam = c.lam32;
  c.p32.eta = c.eta32;
  for (int k = 0; k < 3; ++k) c.Rdd[k] = cv.take<double>(V);
  if (c.adj) {
    c.MB = cv.take<double>(V);
    c.LB = cv.take<double>(V);
    c.EB = cv.take<double>(V);
    c.TB = cv.take<double>(V);
    for (int k = 0; k < 4; ++k) c.T[k] = cv.take<double>(V);
    for (int k = 0; k < 3; ++k) c.Y[k] = cv.take<double>(V);
    c.KB = cv.take<double>(V);
    c.RB = cv.take<double>(V);
    c.IDD = cv.take<double>(V);
    c.DDB = cv.take<double>(V);
    for (int k = 0; k < 6; ++k) c.SLO[k] = cv.take<double>(V);
    c.DB = cv.take<double>(V);
    for (int k = 0; k < 3; ++k) c.VB[k] = cv.take<double>(V);
    c.gs = cv.take<tumor::GradScalars>(1);
  }
  c.sv64 = cv.take<tumor::SolveScalars>(tumor::kMaxSys);
  c.sv32 = cv.take<tumor::SolveScalars>(tumor::kMaxSys);
  c.bflag = cv.take<int>(4);
  c.cs = cv.take<tumor::CoefScalars>(1);
  c.partials = cv.take<double>((size_t)tumor::kPartialsCount);
  c.dpart = cv.take<double>((size_t)tumor::kPartialsCount);
}

size_t workspace_size(const tumor_config& cfg) {
  Ctx c;
  std::memset(&c, 0, sizeof(c));
  c.n = cfg.n;
  c.V = (long long)cfg.n * cfg.n * cfg.n;
  c.S = c.V / 2;
  c.mixed = cfg.precision == TUMOR_PREC_MIXED;
  c.adj = (cfg.flags & TUMOR_F_ADJOINT) != 0;
  Carver cv{nullptr, 0, true};
  layout(c, cv);
  return (cv.off + 255) & ~size_t(255);
}

template <typename R>
PrecBufs<R>& pb(Ctx& c);
template <>
PrecBufs<double>& pb<double>(Ctx& c) { return c.p64; }
template <>
PrecBufs<float>& pb<float>(Ctx& c) { return c.p32; }

// ---------------------------------------------------------- program helpers
struct Prog {
  ColProg p;
  Prog() {
    std::memset(&p, 0, sizeof(p));
  }
  Prog& in(int k, const void* ptr) {
    p.in[k] = ptr;
    return *this;
  }
  Prog& out(void* dst, std::initializer_list<ColTerm> terms, const int* oskip = nullptr) {
    const int o = p.nout++;
    p.out[o] = dst;
    p.oskip[o] = oskip;
    int q = 0;
    for (const ColTerm& t : terms) p.term[o][q++] = t;
    p.nterm[o] = q;
    return *this;
  }
  Prog& skip(const int* s) {
    p.skip = s;
    return *this;
  }
};

XProg to_x(const ColProg& p, double scale) {
  XProg x;
  std::memset(&x, 0, sizeof(x));
  for (int k = 0; k < tumor::kMaxCol; ++k) {
    x.in[k] = p.in[k];
    x.out[k] = p.out[k];
    x.nterm[k] = p.nterm[k];
    for (int q = 0; q < tumor::kMaxTerms; ++q) x.term[k][q] = p.term[k][q];
  }
  x.nout = p.nout;
  x.scale = scale;
  x.skip = p.skip;
  return x;
}

constexpr ColTerm T1(int s, double c = 1.0) { return ColTerm{s, SYM_ONE, c}; }
constexpr ColTerm TW(int s, double c = 1.0) { return ColTerm{s, SYM_IW, c}; }
constexpr ColTerm TR(int s, double c = 1.0) { return ColTerm{s, SYM_RAW, c}; }

// One factor of a physical-space product: C2R of a sum of terms.
struct Fac {
  int n = 0;
  ColTerm t[tumor::kMaxTerms];
};
Fac fac(std::initializer_list<ColTerm> terms) {
  Fac f;
  for (const ColTerm& x : terms) {
    if (f.n == tumor::kMaxTerms) throw std::logic_error("fac: too many terms");
    f.t[f.n++] = x;
  }
  return f;
}

// Builder of a physical-product x pass (XDotArgs).
struct DotProg {
  tumor::XDotArgs a;
  DotProg() { std::memset(&a, 0, sizeof(a)); }
  DotProg& in(int k, const void* ptr) {
    a.in[k] = ptr;
    return *this;
  }
  // a new output: dst = (accumulate: dst +=) the products added after it
  DotProg& out(double* dst, bool accumulate = false) {
    if (a.nout == tumor::kMaxDotOut) throw std::logic_error("DotProg: too many outputs");
    const int o = a.nout++;
    a.out[o] = dst;
    a.accumulate[o] = accumulate ? 1 : 0;
    return *this;
  }
  // coef * C2R(fa) * C2R(fb) into the last output (fb empty: coef * C2R(fa))
  DotProg& prod(double coef, const Fac& fa, const Fac& fb = Fac()) {
    const int o = a.nout - 1;
    if (o < 0 || a.nprod[o] == tumor::kMaxDotProd) throw std::logic_error("DotProg: too many products");
    const int d = a.nprod[o]++;
    a.coef[o][d] = coef;
    put(a.fa[o][d], fa);
    put(a.fb[o][d], fb);
    return *this;
  }
  static void put(tumor::XFactor& f, const Fac& src) {
    f.nterm = src.n;
    for (int q = 0; q < src.n; ++q)
      f.term[q] = tumor::DotTerm{(short)src.t[q].src, (short)src.t[q].sym, (float)src.t[q].coef};
  }
};

// Krylov work fused into an operator apply (see ZPUpdateArgs / ColProg.dsv).
struct Fuse {
  bool pupdate;  // first pass: x += alpha p, p = M^-1 r + beta p (in place) before transforming p
  const void* r;
  void* x;
  tumor::SolveScalars* sv;
  tumor::PrecConsts pc;
};

template <typename R>
void colp(Ctx& c, int axis, bool inv, const Prog& pr) {
  bool used[tumor::kMaxCol] = {false};
  for (int o = 0; o < pr.p.nout; ++o)
    for (int q = 0; q < pr.p.nterm[o]; ++q) used[pr.p.term[o][q].src] = true;
  int nin = 0;
  for (int k = 0; k < tumor::kMaxCol; ++k) nin += used[k] ? 1 : 0;
  // each array once: a dot operand that is also an input is not counted again
  int ndot = 0;
  if (pr.p.dsv)
    for (int o = 0; o < pr.p.nout; ++o) {
      const void* d = pr.p.dotp[o];
      bool seen = d == nullptr;
      for (int k = 0; k < tumor::kMaxCol && !seen; ++k) seen = used[k] && pr.p.in[k] == d;
      for (int q = 0; q < o && !seen; ++q) seen = pr.p.dotp[q] == d;
      ndot += seen ? 0 : 1;
    }
  const double bytes = double(nin + pr.p.nout + ndot) * double(c.V) * sizeof(R);
  // FP32 y and z passes are separate kernel instances (segment widths differ),
  // so they are timed as separate classes; every class is one kernel symbol
  const bool z32 = sizeof(R) == 4 && axis == 2;
  const int cls = inv ? (z32 ? TUMOR_K_COLINV32Z : kcls<R>(TUMOR_K_COLINV64, TUMOR_K_COLINV32))
                      : (pr.p.dsv ? kcls<R>(TUMOR_K_COLDOT64, TUMOR_K_COLDOT32)
                                  : (z32 ? TUMOR_K_COLFWD32Z : kcls<R>(TUMOR_K_COLFWD64, TUMOR_K_COLFWD32)));
  timed(c, cls, bytes,
        [&] { tumor::launch_col_pass<R>(c.n, axis, inv, pr.p, pb<R>(c).tw, c.st); });
}

// Forward 3-D transform of coef_a * a (+ coef_b * b), physical FP64 -> spectral R.
template <typename R>
void fwd3(Ctx& c, const double* a, const double* b, cplx<R>* out, double ca = 1.0, double cb = 1.0) {
  PrecBufs<R>& P = pb<R>(c);
  Prog x;
  x.in(0, a).in(1, b);
  if (b) x.out(P.A[0], {T1(0, ca), T1(1, cb)});
  else x.out(P.A[0], {T1(0, ca)});
  timed(c, TUMOR_K_XOTHER, double(b ? 2 : 1) * c.V * 8.0 + double(c.V) * sizeof(R),
        [&] { tumor::launch_xfwd<R>(c.n, to_x(x.p, 1.0), P.tw, c.st, true); });
  colp<R>(c, 1, false, Prog().in(0, P.A[0]).out(P.B[0], {T1(0)}));
  colp<R>(c, 2, false, Prog().in(0, P.B[0]).out(out, {T1(0)}));
}

// Inverse 3-D transform (spectral R -> physical R) with an optional derivative
// along axis d (0, 1, 2 = x, y, z; -1 = none) and a scale.
template <typename R>
void inv3(Ctx& c, const cplx<R>* in, R* out, double scale, int d = -1) {
  PrecBufs<R>& P = pb<R>(c);
  colp<R>(c, 2, true, Prog().in(0, in).out(P.A[0], {d == 2 ? TW(0) : T1(0)}));
  colp<R>(c, 1, true, Prog().in(0, P.A[0]).out(P.B[0], {d == 1 ? TW(0) : T1(0)}));
  Prog x;
  x.in(0, P.B[0]).out(out, {d == 0 ? TW(0) : T1(0)});
  timed(c, TUMOR_K_XOTHER, 2.0 * c.V * sizeof(R), [&] { tumor::launch_xinv<R>(c.n, to_x(x.p, scale), P.tw, c.st); });
}

// Fused first pass: p = M^-1 r + beta p, then the z-inverse transforms of p
// and i w_z p per component into outs[2a], outs[2a+1].
template <typename R>
void zinv_pupdate(Ctx& c, int ncomp, const Fuse& f, cplx<R>* p, void* const* outs) {
  tumor::ZPUpdateArgs za;
  std::memset(&za, 0, sizeof(za));
  za.r = f.r;
  za.p = p;
  za.x = f.x;
  for (int k = 0; k < 2 * ncomp; ++k) za.out[k] = outs[k];
  za.sv = f.sv;
  za.cs = c.cs;
  za.pc = f.pc;
  // reads r, p, x; writes p, x and the two transformed outputs
  const int cls = ncomp == 3 ? kcls<R>(TUMOR_K_ZINVP64, TUMOR_K_ZINVP32) : kcls<R>(TUMOR_K_ZINVP64_1, TUMOR_K_ZINVP32_1);
  timed(c, cls, 7.0 * ncomp * double(c.V) * sizeof(R),
        [&] { tumor::launch_zinv_pupdate<R>(c.n, ncomp, za, pb<R>(c).tw, c.st); });
}

// out = raw * in + dcoef * D in (spectral), D c = div(K grad c).
template <typename R>
void diff_apply(Ctx& c, const cplx<R>* in, cplx<R>* out, double raw, double dcoef, const int* skip,
                const Fuse* fz = nullptr) {
  PrecBufs<R>& P = pb<R>(c);
  if (fz && fz->pupdate) {
    void* outs[2] = {P.A[0], P.A[1]};
    zinv_pupdate<R>(c, 1, *fz, const_cast<cplx<R>*>(in), outs);
  } else {
    colp<R>(c, 2, true, Prog().in(0, in).out(P.A[0], {T1(0)}).out(P.A[1], {TW(0)}).skip(skip));
  }
  colp<R>(c, 1, true,
          Prog().in(0, P.A[0]).in(1, P.A[1]).out(P.B[0], {T1(0)}).out(P.B[1], {TW(0)}).out(P.B[2], {T1(1)}).skip(
              skip));
  tumor::XDiffArgs xa;
  std::memset(&xa, 0, sizeof(xa));
  xa.in[0] = P.B[0];
  xa.in[1] = P.B[1];
  xa.in[2] = P.B[2];
  xa.out[0] = P.A[0];
  xa.out[1] = P.A[1];
  xa.out[2] = P.A[2];
  xa.K = P.K;
  xa.skip[0] = skip;
  xa.ns = 1;
  timed(c, kcls<R>(TUMOR_K_XDIFF64, TUMOR_K_XDIFF32), 7.0 * c.V * sizeof(R),
        [&] { tumor::launch_xdiff<R>(c.n, xa, P.tw, c.st); });
  colp<R>(c, 1, false,
          Prog().in(0, P.A[0]).in(1, P.A[1]).in(2, P.A[2]).out(P.B[0], {T1(0), TW(1)}).out(P.B[1], {T1(2)}).skip(skip));
  Prog z;
  z.in(0, P.B[0]).in(1, P.B[1]).in(2, in).skip(skip);
  // the untransformed term last: the inner-product pass takes p from it
  if (raw != 0.0) z.out(out, {T1(0, dcoef), TW(1, dcoef), TR(2, raw)});
  else z.out(out, {T1(0, dcoef), TW(1, dcoef)});
  if (fz) {
    z.p.dotp[0] = in;
    z.p.dsv = fz->sv;
    z.p.dpart = c.dpart;
  }
  colp<R>(c, 2, false, z);
}

// out = (eta - L) in on 3-component spectra.
template <typename R>
void elast_apply(Ctx& c, const cplx<R>* in, cplx<R>* out, const int* skip, const Fuse* fz = nullptr) {
  PrecBufs<R>& P = pb<R>(c);
  const long long S = c.S;
  auto** A = P.A;
  auto** B = P.B;
  if (fz && fz->pupdate) {
    void* outs[6] = {A[0], A[3], A[1], A[4], A[2], A[5]};
    zinv_pupdate<R>(c, 3, *fz, const_cast<cplx<R>*>(in), outs);
  } else
  colp<R>(c, 2, true,
          Prog()
              .in(0, in)
              .in(1, in + S)
              .in(2, in + 2 * S)
              .out(A[0], {T1(0)})
              .out(A[3], {TW(0)})
              .out(A[1], {T1(1)})
              .out(A[4], {TW(1)})
              .out(A[2], {T1(2)})
              .out(A[5], {TW(2)})
              .skip(skip));
  Prog y;
  for (int k = 0; k < 6; ++k) y.in(k, A[k]);
  // outputs that share a source are adjacent, so the pass loads each input once
  y.out(B[0], {T1(0)})
      .out(B[3], {TW(0)})
      .out(B[1], {T1(1)})
      .out(B[4], {TW(1)})
      .out(B[2], {T1(2)})
      .out(B[5], {TW(2), T1(4)})
      .out(B[6], {T1(3)})
      .out(B[7], {T1(5)})
      .skip(skip);
  colp<R>(c, 1, true, y);
  tumor::XElastArgs xa;
  for (int k = 0; k < 8; ++k) {
    xa.in[k] = B[k];
    xa.out[k] = A[k];
  }
  xa.mu = P.mu;
  xa.lam = P.lam;
  xa.eta = P.eta;
  xa.skip = skip;
  timed(c, kcls<R>(TUMOR_K_XELAST64, TUMOR_K_XELAST32), 19.0 * c.V * sizeof(R),
        [&] { tumor::launch_xelast<R>(c.n, xa, P.tw, c.st); });
  Prog yf;
  for (int k = 0; k < 8; ++k) yf.in(k, A[k]);
  yf.out(B[0], {T1(0), TW(3, -1.0)})
      .out(B[1], {T1(1), TW(4, -1.0)})
      .out(B[2], {T1(2), TW(5, -1.0)})
      .out(B[3], {T1(6)})
      .out(B[4], {T1(5)})
      .out(B[5], {T1(7)})
      .skip(skip);
  colp<R>(c, 1, false, yf);
  Prog zf;
  for (int k = 0; k < 6; ++k) zf.in(k, B[k]);
  zf.out(out, {T1(0), TW(3, -1.0)})
      .out(out + S, {T1(1), TW(4, -1.0)})
      .out(out + 2 * S, {T1(2), TW(5, -1.0)})
      .skip(skip);
  if (fz) {
    for (int k = 0; k < 3; ++k) zf.p.dotp[k] = in + k * S;
    zf.p.dsv = fz->sv;
    zf.p.dpart = c.dpart;
  }
  colp<R>(c, 2, false, zf);
}

// Spectral right-hand side -b of the elasticity system from tau (physical),
// b = zeta tanh(tau) grad(tau)  (e:forcingfunction).  Written to out (3 S).
void force_rhs(Ctx& c, const double* pa, const double* pbp, cplx<double>* out) {
  PrecBufs<double>& P = c.p64;
  auto** A = P.A;
  auto** B = P.B;
  fwd3<double>(c, pa, pbp, A[1]);
  colp<double>(c, 2, true, Prog().in(0, A[1]).out(B[0], {T1(0)}).out(B[1], {TW(0)}));
  colp<double>(c, 1, true, Prog().in(0, B[0]).in(1, B[1]).out(A[0], {T1(0)}).out(A[1], {TW(0)}).out(A[2], {T1(1)}));
  tumor::XForceArgs xa;
  xa.in[0] = A[0];
  xa.in[1] = A[1];
  xa.in[2] = A[2];
  xa.out[0] = B[0];
  xa.out[1] = B[1];
  xa.out[2] = B[2];
  xa.zeta = c.prm.zeta;
  timed(c, TUMOR_K_XOTHER, 6.0 * c.V * 8.0, [&] { tumor::launch_xforce<double>(c.n, xa, P.tw, c.st); });
  colp<double>(c, 1, false,
               Prog().in(0, B[0]).in(1, B[1]).in(2, B[2]).out(A[0], {T1(0)}).out(A[1], {T1(1)}).out(A[2], {T1(2)}));
  colp<double>(c, 2, false,
               Prog()
                   .in(0, A[0])
                   .in(1, A[1])
                   .in(2, A[2])
                   .out(out, {T1(0)})
                   .out(out + c.S, {T1(1)})
                   .out(out + 2 * c.S, {T1(2)}));
}

// Velocity v = (u^n - u^{n-1}) / dt and its divergence, physical FP64.
void velocity(Ctx& c) {
  PrecBufs<double>& P = c.p64;
  auto** A = P.A;
  auto** B = P.B;
  const long long S = c.S;
  const double idt = 1.0 / c.cfg.dt;
  Prog z;
  for (int k = 0; k < 3; ++k) z.in(k, c.U + k * S).in(3 + k, c.Up + k * S);
  z.out(A[0], {T1(0, idt), T1(3, -idt)})
      .out(A[1], {T1(1, idt), T1(4, -idt)})
      .out(A[2], {T1(2, idt), T1(5, -idt)})
      .out(A[3], {TW(2, idt), TW(5, -idt)});
  colp<double>(c, 2, true, z);
  colp<double>(c, 1, true,
               Prog()
                   .in(0, A[0])
                   .in(1, A[1])
                   .in(2, A[2])
                   .in(3, A[3])
                   .out(B[0], {T1(0)})
                   .out(B[1], {T1(1)})
                   .out(B[2], {T1(2)})
                   .out(B[3], {T1(3), TW(1)}));
  Prog x;
  x.in(0, B[0]).in(1, B[1]).in(2, B[2]).in(3, B[3]);
  x.out(c.vel[0], {T1(0)}).out(c.vel[1], {T1(1)}).out(c.vel[2], {T1(2)}).out(c.vel[3], {TW(0), T1(3)});
  timed(c, TUMOR_K_XOTHER, 8.0 * c.V * 8.0,
        [&] { tumor::launch_xinv<double>(c.n, to_x(x.p, 1.0 / (double)c.V), P.tw, c.st); });
}

// ---------------------------------------------------------------- PCG control
void readback(Ctx& c, tumor::SolveScalars* dev) {
  HIPCHECK(hipMemcpyAsync(c.hsv, dev, sizeof(tumor::SolveScalars), hipMemcpyDeviceToHost, c.st));
  HIPCHECK(hipStreamSynchronize(c.st));
}

struct SolveOut {
  int it = 0;
  int outer = 0;
  double relres = 0.0;
  bool conv = true;
  bool bad = false;
};

template <typename R>
tumor::KrylovArgs kargs(Ctx& c, int ncomp, cplx<R>* x, tumor::SolveScalars* sv, double h, int kind) {
  PrecBufs<R>& P = pb<R>(c);
  tumor::KrylovArgs a;
  std::memset(&a, 0, sizeof(a));
  a.x = x;
  a.r = P.r;
  a.p = P.p;
  a.q = P.q;
  a.b = nullptr;
  a.ax = nullptr;
  a.cs = c.cs;
  a.sv = sv;
  a.partials = c.partials;
  a.n = c.n;
  a.ncomp = ncomp;
  a.pc.h = h;
  a.pc.kind = kind;
  a.scale32 = 1.0;
  return a;
}

// Plain PCG iterations after the residual r and its norms are in place.
// `apply(p, q, skip)` computes q = A p.  Iterations are queued in chunks
// between scalar read-backs: first the predicted count + 1, then the count
// that the residual reduction observed so far (from rr0, ||r||^2 at the
// start) predicts, + 1.  Kernels of an iteration after convergence see the
// device `done` flag and return at once, so the chunking changes only timing.
template <typename R, typename Apply>
int pcg_iterate(Ctx& c, tumor::KrylovArgs a, Apply apply, double thr2, int limit, bool fixed, int pred,
                int zero_x, bool& conv, bool& bad, double rr0) {
  a.thr2 = thr2;
  a.limit = limit;
  a.fixed = fixed ? 1 : 0;
  a.dpart = c.dpart;
  a.dnb = tumor::col_pass_blocks<R>(c.n, 2);
  a.dstride = 1;
  const int kc = kcls<R>(TUMOR_K_KRYLOV64, TUMOR_K_KRYLOV32);
  const double vb = double(a.ncomp) * double(c.V) * sizeof(R);  // one Krylov vector
  timed(c, kc, (zero_x ? 3.0 : 2.0) * vb, [&] { tumor::launch_pcg_start<R>(a, zero_x, c.st); });
  int launched = 0;
  int chunk = fixed ? std::min(limit, 64) : std::max(1, std::min(limit, pred + 1));
  tumor::SolveScalars* sv = a.sv;
  const int* skip = &sv->done;
  for (;;) {
    for (int k = 0; k < chunk && launched < limit; ++k, ++launched) {
      c.cur_tag = launched;
      // iteration k: (p = M^-1 r + beta p fused into the first pass for k > 0),
      // q = A p with alpha = rho / <p, q> fused into the last pass, then x, r
      Fuse fz{launched > 0, a.r, a.x, sv, a.pc};
      apply(static_cast<const cplx<R>*>(a.p), static_cast<cplx<R>*>(a.q), skip, &fz);
      timed(c, kc, 3.0 * vb, [&] { tumor::launch_pcg_update<R>(a, c.st); });
    }
    c.cur_tag = -1;
    HIPCHECK(hipGetLastError());
    readback(c, sv);
    timers_flush(c, c.hsv->it);
    if (c.hsv->done || launched >= limit) break;
    chunk = 4;
    const double rr = c.hsv->rr;
    const int it = c.hsv->it;
    if (fixed) {
      chunk = std::min(limit - launched, 64);
    } else if (rr0 > 0.0 && it > 0 && rr > thr2 && rr < rr0 && std::isfinite(rr)) {
      // mean log reduction per iteration so far; CG does not slow down late
      const double per_it = std::log(rr / rr0) / it;
      const double left = std::log(thr2 / rr) / per_it;
      if (std::isfinite(left)) chunk = std::max(1, std::min(32, (int)std::ceil(left) + 1));
    }
  }
  timed(c, kc, 3.0 * vb, [&] { tumor::launch_pcg_xfinal<R>(a, c.st); });
  conv = c.hsv->conv != 0;
  bad = c.hsv->bad != 0;
  return c.hsv->it;
}

// Solve A x = b for a spectral system.  On entry x holds x0 and `resid0`
// computes r = b - A x0 (and b, norms) into the FP64 vectors.  For the mixed
// precision the FP32 inner PCG corrects x in FP64 outer iterations.
template <typename Apply64, typename Apply32, typename Resid64>
SolveOut solve_system(Ctx& c, int ncomp, int kind, double h, cplx<double>* x, cplx<double>* bvec, double rtol,
                      int which, Apply64 A64, Apply32 A32, Resid64 resid0) {
  SolveOut so;
  tumor::KrylovArgs a = kargs<double>(c, ncomp, x, c.sv64, h, kind);
  a.b = bvec;
  resid0(a);
  readback(c, c.sv64);
  const double bb = c.hsv->bb;
  double rr = c.hsv->rr;
  if (c.hsv->bad) {
    so.bad = true;
    so.conv = false;
    return so;
  }
  const long long cnt = 2LL * ncomp * c.S;  // reals
  if (bb == 0.0) {
    HIPCHECK(hipMemsetAsync(x, 0, cnt * sizeof(double), c.st));
    return so;
  }
  const double thr2 = rtol * rtol * bb;
  int forced = -1;
  if (c.has_forced && which >= 0 && which < 4) forced = c.forced[which];
  if (forced < 0 && rr <= thr2) {
    so.relres = std::sqrt(rr / bb);
    return so;
  }
  const int pred = c.pred[which >= 0 ? which : 3];
  if (!c.mixed) {
    bool conv = true, bad = false;
    const bool fixed = forced >= 0;
    const int limit = fixed ? forced : c.cfg.max_it;
    if (limit > 0) so.it = pcg_iterate<double>(c, a, A64, thr2, limit, fixed, pred, 0, conv, bad, rr);
    so.conv = conv;
    so.bad = bad;
    so.relres = std::sqrt(c.hsv->rr / bb);
    if (which >= 0) c.pred[which] = std::max(1, so.it);
    return so;
  }
  // Mixed precision: x64 += PCG32(b - A64 x64) until the FP64 residual meets rtol.
  PrecBufs<float>& P = c.p32;
  tumor::KrylovArgs a32 = kargs<float>(c, ncomp, P.x, c.sv32, h, kind);
  // r32 = float(r64): rerun the residual kernel on r64 with no subtraction.
  tumor::KrylovArgs conv_args = a;
  conv_args.b = a.r;
  conv_args.ax = nullptr;
  const int max_outer = 30;
  int total = 0;
  while (so.outer < max_outer) {
    // The FP32 copy of the residual is scaled by a power of two that brings its
    // root-mean-square value near 1 (exact, and invisible to PCG's ratios), so
    // that a residual below FP32's range still yields a correction; the
    // correction is unscaled when it is added to x.
    const double rms = std::sqrt(rr / double(cnt));
    const double sc = (rms > 0.0 && std::isfinite(rms)) ? std::ldexp(1.0, -std::ilogb(rms)) : 1.0;
    conv_args.scale32 = sc;
    timed(c, TUMOR_K_KRYLOV64, ncomp * c.V * (16.0 + 4.0), [&] { tumor::launch_residual<double>(conv_args, P.r, c.st); });
    const double need = rtol * std::sqrt(bb / rr);
    const double in_rtol = std::max(1e-4, 0.3 * need);
    bool conv = true, bad = false;
    int inner_it = 0;
    // inner solve with x32 = 0, r32 from above; threshold relative to ||r32||
    tumor::KrylovArgs ai = a32;
    ai.x = P.x;
    const double thr_in = in_rtol * in_rtol * rr * sc * sc;
    int* pin = &c.pred_in[which >= 0 ? which : 3][std::min(so.outer, 2)];
    inner_it = pcg_iterate<float>(c, ai, A32, thr_in, c.cfg.max_it, false, *pin, 1, conv, bad, rr * sc * sc);
    if (conv) *pin = std::max(1, inner_it);
    total += inner_it;
    so.outer++;
    if (bad) {
      so.bad = true;
      so.conv = false;
      break;
    }
    // x64 += x32 / sc: read x64 and x32, write x64
    timed(c, TUMOR_K_KRYLOV64, 20.0 * cnt, [&] { tumor::launch_add32to64(x, P.x, 1.0 / sc, cnt, c.st); });
    // r64 = b - A64 x64
    A64(x, c.p64.q, nullptr);
    tumor::KrylovArgs ar = a;
    ar.b = bvec;
    ar.ax = c.p64.q;
    timed(c, TUMOR_K_KRYLOV64, 3.0 * ncomp * c.V * 8.0, [&] { tumor::launch_residual<double>(ar, nullptr, c.st); });
    readback(c, c.sv64);
    rr = c.hsv->rr;
    if (c.hsv->bad) {
      so.bad = true;
      so.conv = false;
      break;
    }
    if (rr <= thr2) break;
    if (!conv && inner_it >= c.cfg.max_it) break;
  }
  so.it = total;
  so.relres = std::sqrt(rr / bb);
  so.conv = rr <= thr2;
  if (which >= 0) c.pred[which] = std::max(1, total / std::max(1, so.outer));
  return so;
}

// Crank-Nicolson diffusion of the physical field src into dst (may alias).
SolveOut cn_solve(Ctx& c, const double* src, double* dst, int which) {
  const double h = 0.5 * c.cfg.dt;
  cplx<double>* x = c.Un;  // free between elasticity solves
  cplx<double>* b = c.b64;
  fwd3<double>(c, src, nullptr, x);
  auto A64 = [&](const cplx<double>* p, cplx<double>* q, const int* skip, const Fuse* fz = nullptr) {
      diff_apply<double>(c, p, q, 1.0, -h, skip, fz);
    };
  auto A32 = [&](const cplx<float>* p, cplx<float>* q, const int* skip, const Fuse* fz = nullptr) {
      diff_apply<float>(c, p, q, 1.0, -h, skip, fz);
    };
  auto r0 = [&](tumor::KrylovArgs& a) {
    diff_apply<double>(c, x, c.p64.q, 0.0, 1.0, nullptr);
    timed(c, TUMOR_K_KRYLOV64, 4.0 * c.V * 8.0, [&] { tumor::launch_cn_residual<double>(a, x, c.p64.q, c.st); });
  };
  SolveOut so = solve_system(c, 1, tumor::PREC_DIFF, h, x, b, c.cfg.rtol_diff, which, A64, A32, r0);
  inv3<double>(c, x, dst, 1.0 / (double)c.V);
  return so;
}

// ------------------------------------------------ batched CN solves (i, o, l)
// The Crank-Nicolson systems of the species share the operator (1 - dt/2 D_K)
// and its preconditioner, so they are solved as one Krylov iteration over ns
// blocks with per-system scalars and stopping rules (BatchArgs): each FFT
// pass handles every system still iterating (K is read once), and one scalar
// read-back serves all of them.  Each system's arithmetic, sums included, is
// that of its own solve.

template <typename R>
tumor::BatchArgs bargs(Ctx& c, int ns, int active, cplx<R>* x, tumor::SolveScalars* sv, double h) {
  PrecBufs<R>& P = pb<R>(c);
  tumor::BatchArgs a;
  std::memset(&a, 0, sizeof(a));
  a.x = x;
  a.r = P.r;
  a.p = P.p;
  a.q = P.q;
  a.cs = c.cs;
  a.sv = sv;
  a.partials = c.partials;
  a.n = c.n;
  a.ns = ns;
  a.active = active;
  a.pc.h = h;
  a.pc.kind = tumor::PREC_DIFF;
  for (int k = 0; k < tumor::kMaxSys; ++k) a.scale32[k] = 1.0;
  return a;
}

// Krylov work fused into a batched apply (see ZPUpdateArgs.nsys, ColProg.dot_nsys).
struct BFuse {
  bool pupdate;
  const void* r;
  void* x;
  tumor::SolveScalars* sv;  // ns entries
  tumor::PrecConsts pc;
};

// Keeps the timers' batched-apply accounting set for a scope.
struct BatchScope {
  Ctx& c;
  BatchScope(Ctx& cc, int total, int active) : c(cc) {
    c.bsys_total = total;
    c.bsys_active = active;
  }
  ~BatchScope() {
    c.bsys_total = 0;
    c.bsys_active = 0;
  }
};

// out_k = raw * in_k + dcoef * D in_k (spectral) for the ns systems whose
// skip flag is clear; D c = div(K grad c).  Pass buffers: the z inverse into
// 0 .. 2ns-1, the y inverse into 6 .. 6+3ns-1, the x pass in place, the y
// forward into 0 .. 2ns-1.
template <typename R>
void diff_apply_b(Ctx& c, int ns, const cplx<R>* in, cplx<R>* out, double raw, double dcoef,
                  const int* const* skip, const BFuse* fz = nullptr) {
  PrecBufs<R>& P = pb<R>(c);
  cplx<R>* buf[16];
  for (int k = 0; k < 8; ++k) {
    buf[k] = P.A[k];
    buf[8 + k] = P.B[k];
  }
  const long long S = c.S;
  if (fz && fz->pupdate) {
    tumor::ZPUpdateArgs za;
    std::memset(&za, 0, sizeof(za));
    za.r = fz->r;
    za.p = const_cast<cplx<R>*>(in);
    za.x = fz->x;
    for (int k = 0; k < 2 * ns; ++k) za.out[k] = buf[k];
    za.sv = fz->sv;
    za.cs = c.cs;
    za.pc = fz->pc;
    za.nsys = ns;
    timed(c, kcls<R>(TUMOR_K_ZINVPB64, TUMOR_K_ZINVPB32), 7.0 * ns * double(c.V) * sizeof(R),
          [&] { tumor::launch_zinv_pupdate<R>(c.n, 1, za, P.tw, c.st); });
  } else {
    Prog z;
    for (int k = 0; k < ns; ++k) z.in(k, in + k * S).out(buf[2 * k], {T1(k)}, skip[k]).out(buf[2 * k + 1], {TW(k)}, skip[k]);
    colp<R>(c, 2, true, z);
  }
  Prog y;
  for (int k = 0; k < ns; ++k)
    y.in(2 * k, buf[2 * k])
        .in(2 * k + 1, buf[2 * k + 1])
        .out(buf[6 + 3 * k], {T1(2 * k)}, skip[k])
        .out(buf[7 + 3 * k], {TW(2 * k)}, skip[k])
        .out(buf[8 + 3 * k], {T1(2 * k + 1)}, skip[k]);
  colp<R>(c, 1, true, y);
  tumor::XDiffArgs xa;
  std::memset(&xa, 0, sizeof(xa));
  for (int e = 0; e < 3 * ns; ++e) xa.in[e] = xa.out[e] = buf[6 + e];
  for (int k = 0; k < ns; ++k) xa.skip[k] = skip[k];
  xa.K = P.K;
  xa.ns = ns;
  // K once, then three rows in and three out per system
  timed_b(c, kcls<R>(TUMOR_K_XDIFF64, TUMOR_K_XDIFF32), double(c.V) * sizeof(R), 6.0 * double(c.V) * sizeof(R),
          [&] { tumor::launch_xdiff<R>(c.n, xa, P.tw, c.st); });
  Prog yf;
  for (int k = 0; k < ns; ++k)
    yf.in(3 * k, buf[6 + 3 * k])
        .in(3 * k + 1, buf[7 + 3 * k])
        .in(3 * k + 2, buf[8 + 3 * k])
        .out(buf[2 * k], {T1(3 * k), TW(3 * k + 1)}, skip[k])
        .out(buf[2 * k + 1], {T1(3 * k + 2)}, skip[k]);
  colp<R>(c, 1, false, yf);
  Prog zf;
  for (int k = 0; k < ns; ++k) {
    zf.in(3 * k, buf[2 * k]).in(3 * k + 1, buf[2 * k + 1]).in(3 * k + 2, in + k * S);
    // the untransformed term last: the inner-product pass takes p from it
    if (raw != 0.0)
      zf.out(out + k * S, {T1(3 * k, dcoef), TW(3 * k + 1, dcoef), TR(3 * k + 2, raw)}, skip[k]);
    else
      zf.out(out + k * S, {T1(3 * k, dcoef), TW(3 * k + 1, dcoef)}, skip[k]);
  }
  if (fz) {
    for (int k = 0; k < ns; ++k) zf.p.dotp[k] = in + k * S;
    zf.p.dsv = fz->sv;
    zf.p.dpart = c.dpart;
    zf.p.dot_nsys = ns;
  }
  colp<R>(c, 2, false, zf);
}

// Batched PCG iterations after the residuals and norms are in place, for
// the systems in `active`; per system thr2, limit, fixed and pred.  Chunked
// between read-backs like pcg_iterate, on the slowest system's prediction.
template <typename R>
void pcg_iterate_b(Ctx& c, tumor::BatchArgs a, const double* thr2, const int* limit, const bool* fixed,
                   const int* pred, int zero_x, const double* rr0, int* its, bool* conv, bool* bad) {
  const int ns = a.ns;
  int lim_max = 0, chunk = 1;
  bool any_fixed = false;
  for (int k = 0; k < ns; ++k) {
    a.thr2[k] = thr2[k];
    a.limit[k] = limit[k];
    a.fixed[k] = fixed[k] ? 1 : 0;
    its[k] = 0;
    conv[k] = true;
    bad[k] = false;
    if (!(a.active & (1 << k))) continue;
    lim_max = std::max(lim_max, limit[k]);
    any_fixed = any_fixed || fixed[k];
    chunk = std::max(chunk, std::min(limit[k], pred[k] + 1));
  }
  if (any_fixed) chunk = std::min(lim_max, 64);
  a.dpart = c.dpart;
  a.dnb = tumor::col_pass_blocks<R>(c.n, 2);
  const int kc = kcls<R>(TUMOR_K_KRYLOV64, TUMOR_K_KRYLOV32);
  const double vb = double(c.V) * sizeof(R);  // one system's Krylov vector
  const int nact = __builtin_popcount((unsigned)a.active);
  timed(c, kc, (zero_x ? 3.0 : 2.0) * vb * nact, [&] { tumor::launch_bpcg_start<R>(a, zero_x, c.st); });
  const int* skip[tumor::kMaxSys] = {};
  for (int k = 0; k < ns; ++k) skip[k] = &a.sv[k].done;
  {
  BatchScope scope(c, ns, nact);
  c.batch_ns = ns;
  int launched = 0;
  for (;;) {
    for (int i = 0; i < chunk && launched < lim_max; ++i, ++launched) {
      c.cur_tag = launched;
      BFuse fz{launched > 0, a.r, a.x, a.sv, a.pc};
      diff_apply_b<R>(c, ns, static_cast<const cplx<R>*>(a.p), static_cast<cplx<R>*>(a.q), 1.0, -a.pc.h, skip,
                      &fz);
      timed_b(c, kc, 0.0, 3.0 * vb, [&] { tumor::launch_bpcg_update<R>(a, c.st); });
    }
    c.cur_tag = -1;
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(c.hsv, a.sv, ns * sizeof(tumor::SolveScalars), hipMemcpyDeviceToHost, c.st));
    HIPCHECK(hipStreamSynchronize(c.st));
    bool all_done = true;
    int left = 0;
    for (int k = 0; k < ns; ++k) {
      c.batch_it[k] = (a.active & (1 << k)) ? c.hsv[k].it : 0;
      if (!(a.active & (1 << k)) || c.hsv[k].done) continue;
      all_done = false;
      // the remaining iterations the residual reduction of this system predicts
      int more = 4;
      const double rr = c.hsv[k].rr;
      const int it = c.hsv[k].it;
      if (fixed[k]) {
        more = limit[k] - it;
      } else if (rr0[k] > 0.0 && it > 0 && rr > thr2[k] && rr < rr0[k] && std::isfinite(rr)) {
        const double per_it = std::log(rr / rr0[k]) / it;
        const double rest = std::log(thr2[k] / rr) / per_it;
        if (std::isfinite(rest)) more = std::max(1, std::min(32, (int)std::ceil(rest) + 1));
      }
      left = std::max(left, std::min(more, limit[k] - it));
    }
    timers_flush(c, 0x7fffffff);
    if (all_done || launched >= lim_max) break;
    chunk = std::max(1, std::min(left, any_fixed ? 64 : 32));
  }
  c.batch_ns = 0;
  }
  timed(c, kc, 3.0 * vb * nact, [&] { tumor::launch_bpcg_xfinal<R>(a, c.st); });
  for (int k = 0; k < ns; ++k) {
    if (!(a.active & (1 << k))) continue;
    its[k] = c.hsv[k].it;
    conv[k] = c.hsv[k].conv != 0;
    bad[k] = c.hsv[k].bad != 0;
  }
}

// Crank-Nicolson diffusion of ns physical fields src[k] into dst[k] (may
// alias), which[k] = solve slot (iteration predictions, forced counts).
// With rhs set (the adjoint's solves) src[k] are instead right-hand sides:
// (1 - dt/2 D) y_k = src[k] from y_k = 0, and the solutions stay spectral in
// the blocks of Un (dst unused).
void cn_solve_b(Ctx& c, int ns, const double* const* src, double* const* dst, const int* which, SolveOut* so,
                bool rhs = false) {
  const double h = 0.5 * c.cfg.dt;
  const long long S = c.S;
  const int all = (1 << ns) - 1;
  cplx<double>* x = c.Un;  // ns blocks; free between elasticity solves
  for (int k = 0; k < ns; ++k) {
    so[k] = SolveOut();
    fwd3<double>(c, src[k], nullptr, rhs ? c.b64 + k * S : x + k * S);
  }
  PrecBufs<double>& P = c.p64;
  tumor::BatchArgs a = bargs<double>(c, ns, all, x, c.sv64, h);
  a.b = c.b64;
  const int* flag[tumor::kMaxSys] = {};
  for (int k = 0; k < ns; ++k) flag[k] = c.bflag + k;
  auto apply64 = [&](int mask, const cplx<double>* in, cplx<double>* out, double raw, double dcoef) {
    BatchScope scope(c, ns, __builtin_popcount((unsigned)mask));
    tumor::launch_set_flags(c.bflag, ns, mask, c.st);
    diff_apply_b<double>(c, ns, in, out, raw, dcoef, flag);
  };
  if (rhs) {
    // x0 = 0: r = b
    HIPCHECK(hipMemsetAsync(x, 0, ns * S * sizeof(cplx<double>), c.st));
    timed(c, TUMOR_K_KRYLOV64, 2.0 * ns * c.V * 8.0, [&] { tumor::launch_bresidual<double>(a, nullptr, c.st); });
  } else {
    // D x0 for every system, then b = x0 + h D x0 and r = b - (x0 - h D x0)
    apply64(all, x, P.q, 0.0, 1.0);
    timed(c, TUMOR_K_KRYLOV64, 4.0 * ns * c.V * 8.0, [&] { tumor::launch_bcn_residual<double>(a, x, P.q, c.st); });
  }
  HIPCHECK(hipMemcpyAsync(c.hsv, c.sv64, ns * sizeof(tumor::SolveScalars), hipMemcpyDeviceToHost, c.st));
  HIPCHECK(hipStreamSynchronize(c.st));
  double bb[tumor::kMaxSys], rr[tumor::kMaxSys], thr2[tumor::kMaxSys];
  int forced[tumor::kMaxSys];
  int active = 0;
  for (int k = 0; k < ns; ++k) {
    bb[k] = c.hsv[k].bb;
    rr[k] = c.hsv[k].rr;
    thr2[k] = c.cfg.rtol_diff * c.cfg.rtol_diff * bb[k];
    forced[k] = (c.has_forced && which[k] >= 0 && which[k] < 4) ? c.forced[which[k]] : -1;
    if (c.hsv[k].bad) {
      so[k].bad = true;
      so[k].conv = false;
    } else if (bb[k] == 0.0) {
      HIPCHECK(hipMemsetAsync(x + k * S, 0, S * sizeof(cplx<double>), c.st));
    } else if (forced[k] < 0 && rr[k] <= thr2[k]) {
      so[k].relres = std::sqrt(rr[k] / bb[k]);
    } else {
      active |= 1 << k;
    }
  }
  if (!c.mixed) {
    int limit[tumor::kMaxSys], pred[tumor::kMaxSys], its[tumor::kMaxSys];
    bool fixed[tumor::kMaxSys], conv[tumor::kMaxSys], bad[tumor::kMaxSys];
    for (int k = 0; k < ns; ++k) {
      fixed[k] = forced[k] >= 0;
      limit[k] = fixed[k] ? forced[k] : c.cfg.max_it;
      pred[k] = c.pred[which[k]];
      if ((active & (1 << k)) && limit[k] <= 0) {
        // no iterations (a forced count of zero)
        active &= ~(1 << k);
        so[k].relres = std::sqrt(rr[k] / bb[k]);
        c.pred[which[k]] = 1;
      }
    }
    if (active) {
      tumor::BatchArgs ai = a;
      ai.active = active;
      pcg_iterate_b<double>(c, ai, thr2, limit, fixed, pred, 0, rr, its, conv, bad);
      for (int k = 0; k < ns; ++k) {
        if (!(active & (1 << k))) continue;
        so[k].it = its[k];
        so[k].conv = conv[k];
        so[k].bad = bad[k];
        so[k].relres = std::sqrt(c.hsv[k].rr / bb[k]);
        c.pred[which[k]] = std::max(1, its[k]);
      }
    }
  } else {
    // x64 += PCG32(b - A64 x64) per system until its FP64 residual meets rtol
    PrecBufs<float>& Q = c.p32;
    tumor::BatchArgs a32 = bargs<float>(c, ns, 0, Q.x, c.sv32, h);
    const long long cnt = 2LL * S;  // reals per system
    const int max_outer = 30;
    int total[tumor::kMaxSys] = {0, 0, 0};
    while (active) {
      double sc[tumor::kMaxSys] = {1.0, 1.0, 1.0}, thr_in[tumor::kMaxSys], rr_in[tumor::kMaxSys];
      int limit[tumor::kMaxSys], pred[tumor::kMaxSys], its[tumor::kMaxSys];
      bool fixed[tumor::kMaxSys] = {false, false, false}, conv[tumor::kMaxSys], bad[tumor::kMaxSys];
      tumor::BatchArgs cv = a;  // r32 = float(scale * r64), r64 unchanged
      cv.b = a.r;
      cv.ax = nullptr;
      cv.active = active;
      for (int k = 0; k < ns; ++k) {
        limit[k] = c.cfg.max_it;
        thr_in[k] = 0.0;
        rr_in[k] = 0.0;
        pred[k] = 1;
        if (!(active & (1 << k))) continue;
        const double rms = std::sqrt(rr[k] / double(cnt));
        sc[k] = (rms > 0.0 && std::isfinite(rms)) ? std::ldexp(1.0, -std::ilogb(rms)) : 1.0;
        const double need = c.cfg.rtol_diff * std::sqrt(bb[k] / rr[k]);
        const double in_rtol = std::max(1e-4, 0.3 * need);
        thr_in[k] = in_rtol * in_rtol * rr[k] * sc[k] * sc[k];
        rr_in[k] = rr[k] * sc[k] * sc[k];
        pred[k] = c.pred_in[which[k]][std::min(so[k].outer, 2)];
        cv.scale32[k] = sc[k];
      }
      timed(c, TUMOR_K_KRYLOV64, __builtin_popcount((unsigned)active) * c.V * (16.0 + 4.0),
            [&] { tumor::launch_bresidual<double>(cv, Q.r, c.st); });
      tumor::BatchArgs ai = a32;
      ai.active = active;
      pcg_iterate_b<float>(c, ai, thr_in, limit, fixed, pred, 1, rr_in, its, conv, bad);
      double inv_sc[tumor::kMaxSys] = {1.0, 1.0, 1.0};
      int stop = 0;
      for (int k = 0; k < ns; ++k) {
        if (!(active & (1 << k))) continue;
        if (conv[k]) c.pred_in[which[k]][std::min(so[k].outer, 2)] = std::max(1, its[k]);
        total[k] += its[k];
        so[k].outer++;
        inv_sc[k] = 1.0 / sc[k];
        if (bad[k]) {
          so[k].bad = true;
          so[k].conv = false;
          stop |= 1 << k;
        } else if (!conv[k] && its[k] >= c.cfg.max_it) {
          stop |= 1 << k;  // the correction is still added; the FP64 residual decides conv
        }
      }
      // every system that ran without a breakdown adds its correction
      int add = 0;
      for (int k = 0; k < ns; ++k)
        if ((active & (1 << k)) && !so[k].bad) add |= 1 << k;
      timed_b(c, TUMOR_K_KRYLOV64, 20.0 * cnt * __builtin_popcount((unsigned)add), 0.0,
              [&] { tumor::launch_badd32to64(x, Q.x, inv_sc, ns, add, cnt, c.st); });
      // r64 = b - A64 x64 for the systems that added a correction
      if (add) {
        apply64(add, x, P.q, 1.0, -h);
        tumor::BatchArgs ar = a;
        ar.b = c.b64;
        ar.ax = P.q;
        ar.active = add;
        timed(c, TUMOR_K_KRYLOV64, 3.0 * __builtin_popcount((unsigned)add) * c.V * 8.0,
              [&] { tumor::launch_bresidual<double>(ar, nullptr, c.st); });
        HIPCHECK(hipMemcpyAsync(c.hsv, c.sv64, ns * sizeof(tumor::SolveScalars), hipMemcpyDeviceToHost, c.st));
        HIPCHECK(hipStreamSynchronize(c.st));
      }
      int next = 0;
      for (int k = 0; k < ns; ++k) {
        if (!(active & (1 << k))) continue;
        if (so[k].bad) continue;
        rr[k] = c.hsv[k].rr;
        if (c.hsv[k].bad) {
          so[k].bad = true;
          so[k].conv = false;
          continue;
        }
        if (rr[k] <= thr2[k]) continue;                // converged
        if (stop & (1 << k)) continue;                 // inner limit reached without convergence
        if (so[k].outer >= max_outer) continue;
        next |= 1 << k;
      }
      active = next;
    }
    for (int k = 0; k < ns; ++k) {
      if (so[k].outer == 0) continue;
      so[k].it = total[k];
      so[k].relres = std::sqrt(rr[k] / bb[k]);
      so[k].conv = !so[k].bad && rr[k] <= thr2[k];
      c.pred[which[k]] = std::max(1, total[k] / std::max(1, so[k].outer));
    }
  }
  if (!rhs)
    for (int k = 0; k < ns; ++k) inv3<double>(c, x + k * S, dst[k], 1.0 / (double)c.V);
}

// Elasticity solve (eta - L) u = rhs, rhs spectral in b64, warm start from U.
SolveOut elast_solve(Ctx& c, cplx<double>* x, int which) {
  HIPCHECK(hipMemcpyAsync(x, c.U, 3 * c.S * sizeof(cplx<double>), hipMemcpyDeviceToDevice, c.st));
  auto A64 = [&](const cplx<double>* p, cplx<double>* q, const int* skip, const Fuse* fz = nullptr) {
    elast_apply<double>(c, p, q, skip, fz);
  };
  auto A32 = [&](const cplx<float>* p, cplx<float>* q, const int* skip, const Fuse* fz = nullptr) {
    elast_apply<float>(c, p, q, skip, fz);
  };
  auto r0 = [&](tumor::KrylovArgs& a) {
    elast_apply<double>(c, x, c.p64.q, nullptr);
    a.ax = c.p64.q;
    timed(c, TUMOR_K_KRYLOV64, 9.0 * c.V * 8.0, [&] { tumor::launch_residual<double>(a, nullptr, c.st); });
    a.ax = nullptr;
  };
  return solve_system(c, 3, tumor::PREC_ELAST, 0.0, x, c.b64, c.cfg.rtol_elast, which, A64, A32, r0);
}

void refresh(Ctx& c, int do_reaction, const double* const* in, double* const* out) {
  tumor::ReactArgs a;
  std::memset(&a, 0, sizeof(a));
  a.p = in[0];
  a.i_dag = in[1];
  a.i_dd = in[2];
  a.n = in[3];
  a.g = in[4];
  a.w = in[5];
  a.o = in[6];
  a.l = in[7];
  a.f = in[8];
  a.po = out[0];
  a.io = out[1];
  a.no = out[2];
  a.go = out[3];
  a.wo = out[4];
  a.oo = out[5];
  a.lo = out[6];
  a.fo = out[7];
  a.K = c.K;
  a.rho = c.rho;
  a.mu = c.mu;
  a.lam = c.lam;
  a.eta = c.eta;
  a.bg = c.BG;
  a.K32 = c.K32;
  a.mu32 = c.mu32;
  a.lam32 = c.lam32;
  a.eta32 = c.eta32;
  a.cs = c.cs;
  a.partials = c.partials;
  a.V = c.V;
  a.do_reaction = do_reaction;
  a.single = c.single ? 1 : 0;
  a.rc = c.rc;
  a.fc = c.fc;
  const double rb = do_reaction ? (10.0 + 13.0) * c.V * 8.0 + (c.K32 ? 16.0 * c.V : 0.0) : 12.0 * c.V * 8.0;
  timed(c, TUMOR_K_REACT, rb, [&] { tumor::launch_react(a, c.st); });
}

void refresh_state(Ctx& c) {
  enum { P, I, N, O, L, G, W, F };
  const double* in[9] = {c.F[P], c.F[I], c.F[I], c.F[N], c.F[G], c.F[W], c.F[O], c.F[L], c.F[F]};
  double* out[8] = {nullptr};
  refresh(c, 0, in, out);
}

void set_consts(Ctx& c) {
  const tumor_params& p = c.prm;
  auto mu_of = [](double E, double nu) { return E / (2.0 * (1.0 + nu)); };
  auto la_of = [](double E, double nu) { return nu * E / ((1.0 - 2.0 * nu) * (1.0 + nu)); };
  const double s = p.lame_scale;
  c.fc.k_w = p.k_w;
  c.fc.k_g = p.k_g;
  c.fc.k_f = p.k_f;
  c.fc.rho_w = p.rho_w;
  c.fc.rho_g = p.rho_g;
  c.fc.mu_w = s * mu_of(p.E_wm, p.nu_wm);
  c.fc.mu_g = s * mu_of(p.E_gm, p.nu_gm);
  c.fc.mu_f = s * mu_of(p.E_csf, p.nu_csf);
  c.fc.mu_t = s * mu_of(p.E_tumor, p.nu_tumor);
  c.fc.la_w = s * la_of(p.E_wm, p.nu_wm);
  c.fc.la_g = s * la_of(p.E_gm, p.nu_gm);
  c.fc.la_f = s * la_of(p.E_csf, p.nu_csf);
  c.fc.la_t = s * la_of(p.E_tumor, p.nu_tumor);
  c.fc.eta_t = p.eta_tumor;
  c.fc.eta_h = p.eta_healthy;
  c.fc.mu_b = s * mu_of(p.E_bg, p.nu_bg);
  c.fc.la_b = s * la_of(p.E_bg, p.nu_bg);
  c.fc.eta_b = p.eta_bg;
  c.rc.dt = c.cfg.dt;
  c.rc.alpha0 = p.alpha0;
  c.rc.beta0 = p.beta0;
  c.rc.gamma = p.gamma;
  c.rc.sigma_b = p.sigma_b;
  c.rc.o_hyp = p.o_hyp;
  c.rc.o_inv = p.o_inv;
  c.rc.o_mit = 0.5 * (p.o_hyp + p.o_inv);
  c.rc.o_heal = p.o_heal;
  c.rc.delta_s = p.delta_s;
  c.rc.delta_p = p.delta_p;
  c.rc.delta_e = p.delta_e;
  c.rc.delta_half = p.delta_half;
  c.rc.delta_l = p.delta_l;
  c.rc.eps = p.heaviside_eps;
  c.rc.rho_inv_frac = p.rho_inv_frac;
  c.rc.edema = (c.flags & TUMOR_F_EDEMA) ? 1 : 0;
}

int check_params(const tumor_params* p) {
  if (!p) return TUMOR_EINVAL;
  const double* v = reinterpret_cast<const double*>(p);
  for (size_t k = 0; k < sizeof(tumor_params) / sizeof(double); ++k)
    if (!std::isfinite(v[k])) return TUMOR_EINVAL;
  if (!(p->heaviside_eps > 0.0)) return TUMOR_EINVAL;
  if (!(p->o_inv > p->o_hyp)) return TUMOR_EINVAL;  // o_mit strictly below o_inv
  const double nus[5] = {p->nu_wm, p->nu_gm, p->nu_csf, p->nu_tumor, p->nu_bg};
  for (double nu : nus)
    if (!(nu > -1.0 && nu < 0.5)) return TUMOR_EINVAL;
  if (p->eta_tumor < 0.0 || p->eta_healthy < 0.0 || p->eta_bg < 0.0) return TUMOR_EINVAL;
  // e:screening: without any screening the elasticity operator vanishes on the
  // modes whose derivative symbols are all zero, and the force has content there
  if (p->eta_tumor == 0.0 && p->eta_healthy == 0.0 && p->eta_bg == 0.0) return TUMOR_EINVAL;
  return TUMOR_OK;
}

void twiddles(Ctx& c) {
  const int n = c.n;
  // n <= 512 (check_cfg): the tables live on the stack, so that context set-up
  // needs no host heap either
  cplx<double> t64[512];
  cplx<float> t32[512];
  for (int m = 0; m < n; ++m) {
    const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)n;
    t64[m] = {(double)cosl(ang), (double)sinl(ang)};
    t32[m] = {(float)cosl(ang), (float)sinl(ang)};
  }
  HIPCHECK(hipMemcpyAsync(c.p64.tw, t64, n * sizeof(cplx<double>), hipMemcpyHostToDevice, c.st));
  HIPCHECK(hipMemcpyAsync(c.p32.tw, t32, n * sizeof(cplx<float>), hipMemcpyHostToDevice, c.st));
  HIPCHECK(hipStreamSynchronize(c.st));
}

// S1 (Sec. 3): velocity u_t^n = (u^n - u^{n-1}) / dt and its divergence
// (unless `fresh_velocity` is false: the second half-step of the symmetric
// form reuses them), then the semi-Lagrangian step over frac * dt of
// ins[0..5] = p, i, n, g, w, f into outs[0..5].  max |frac dt v| / h lands in
// cs->cfl_bits.
void transport(Ctx& c, const double* const (&ins)[6], double* const (&outs)[6], double frac = 1.0,
               bool fresh_velocity = true) {
  if (fresh_velocity) velocity(c);
  tumor::SLArgs s;
  s.vx = c.vel[0];
  s.vy = c.vel[1];
  s.vz = c.vel[2];
  s.div = c.vel[3];
  s.p = ins[0];
  s.i = ins[1];
  s.n = ins[2];
  s.g = ins[3];
  s.w = ins[4];
  s.f = ins[5];
  s.po = outs[0];
  s.io = outs[1];
  s.no = outs[2];
  s.go = outs[3];
  s.wo = outs[4];
  s.fo = outs[5];
  s.n_grid = c.n;
  s.dt = frac * c.cfg.dt;
  s.s = frac * c.cfg.dt / (2.0 * M_PI / c.n);
  // the tiled step reads v (3), div v and the six fields once and writes six
  // fields (16 FP64 arrays); FP32 adds the scan for the scales (6 FP64 reads)
  HIPCHECK(hipMemsetAsync(&c.cs->cfl_bits, 0, 7 * sizeof(unsigned long long), c.st));  // cfl + qmax[6]
  timed(c, TUMOR_K_SL, (c.mixed ? 22.0 : 16.0) * 8.0 * c.V, [&] {
    if (c.mixed) tumor::launch_sl_tile<float>(s, c.cs, c.st);
    else tumor::launch_sl_tile<double>(s, c.cs, c.st);
  });
}

// Sub-step boundary k (0..5): an event for the sub-step timer and a roctx
// range (named for the sub-step that starts here) for profilers.
void substep_mark(Ctx& c, int k) {
  static const char* const names[6] = {"tumor transport", "tumor diffusion", "tumor reaction",
                                       "tumor transport (second half)", "tumor elasticity", ""};
  if (k > 0) roctxRangePop();
  if (k < 5) roctxRangePushA(names[k]);
  if (c.sub_on) HIPCHECK(hipEventRecord(c.sub_ev[k], c.st));
}

void do_step(Ctx& c, tumor_step_stats* stats, int& status) {
  enum { P, I, N, O, L, G, W, F };
  const int n = c.n;
  (void)n;
  // Symmetric form: S1 over dt/2 here and again after the reaction.
  const bool strang = (c.flags & TUMOR_F_STRANG) && (c.flags & TUMOR_F_ADVECTION);
  substep_mark(c, 0);
  // S1: transport with u_t^n = (u^n - u^{n-1}) / dt
  if (c.flags & TUMOR_F_ADVECTION) {
    const double* const ins[6] = {c.F[P], c.F[I], c.F[N], c.F[G], c.F[W], c.F[F]};
    double* const outs[6] = {c.G[P], c.G[I], c.G[N], c.G[G], c.G[W], c.G[F]};
    transport(c, ins, outs, strang ? 0.5 : 1.0);
    if (strang) {
      // coefficients (and their means) of the half-transported state
      const double* in[9] = {c.G[P], c.G[I], c.G[I], c.G[N], c.G[G], c.G[W], c.F[O], c.F[L], c.G[F]};
      double* out[8] = {nullptr};
      refresh(c, 0, in, out);
    }
  } else {
    const int ids[6] = {P, I, N, G, W, F};
    for (int k : ids)
      HIPCHECK(hipMemcpyAsync(c.G[k], c.F[k], c.V * sizeof(double), hipMemcpyDeviceToDevice, c.st));
  }
  SolveOut sd[3];
  substep_mark(c, 1);
  if (c.single) {
    // Single-species model: CN diffusion of c, then its reaction and the refresh.
    sd[0] = cn_solve(c, c.G[P], c.Rdd[0], 0);
    substep_mark(c, 2);
    const double* in[9] = {c.G[P], c.G[P], c.Rdd[0], c.G[N], c.G[G], c.G[W], c.F[O], c.F[L], c.G[F]};
    double* out[8] = {c.F[P], c.F[I], c.F[N], c.F[G], c.F[W], c.F[O], c.F[L], c.F[F]};
    refresh(c, 1, in, out);
  } else {
  // S2: Crank-Nicolson diffusion of i, o (and l), one batched solve.
  {
    const double* src[3] = {c.G[I], c.F[O], c.F[L]};
    double* dst[3] = {c.Rdd[0], c.Rdd[1], c.Rdd[2]};
    const int which[3] = {0, 1, 2};
    cn_solve_b(c, (c.flags & TUMOR_F_EDEMA) ? 3 : 2, src, dst, which, sd);
  }
  if (!(c.flags & TUMOR_F_EDEMA))
    HIPCHECK(hipMemcpyAsync(c.Rdd[2], c.F[L], c.V * sizeof(double), hipMemcpyDeviceToDevice, c.st));
  substep_mark(c, 2);
  // S3-S5: reaction, oxygen, edema, refresh.
  {
    const double* in[9] = {c.G[P], c.G[I], c.Rdd[0], c.G[N], c.G[G], c.G[W], c.Rdd[1], c.Rdd[2], c.G[F]};
    double* out[8] = {c.F[P], c.F[I], c.F[N], c.F[G], c.F[W], c.F[O], c.F[L], c.F[F]};
    refresh(c, 1, in, out);
  }
  }
  substep_mark(c, 3);
  if (strang) {
    // second half-step of S1 with the same velocity, from F back into G; the
    // two sets swap roles so the state stays in F; then the refresh (S5)
    const double* const ins[6] = {c.F[P], c.F[I], c.F[N], c.F[G], c.F[W], c.F[F]};
    double* const outs[6] = {c.G[P], c.G[I], c.G[N], c.G[G], c.G[W], c.G[F]};
    transport(c, ins, outs, 0.5, false);
    for (int k : {P, I, N, G, W, F}) std::swap(c.F[k], c.G[k]);
    refresh_state(c);
  }
  // S6-S7: elasticity and rotation.
  substep_mark(c, 4);
  SolveOut se;
  if (c.flags & TUMOR_F_ELASTICITY) {
    force_rhs(c, c.F[P], c.F[N], c.b64);
    se = elast_solve(c, c.Un, 3);
    cplx<double>* old = c.Up;
    c.Up = c.U;
    c.U = c.Un;
    c.Un = old;
  } else {
    HIPCHECK(hipMemcpyAsync(c.Up, c.U, 3 * c.S * sizeof(cplx<double>), hipMemcpyDeviceToDevice, c.st));
  }
  substep_mark(c, 5);
  c.has_forced = false;
  timers_flush(c, 0x7fffffff);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipMemcpyAsync(c.hcs, c.cs, sizeof(tumor::CoefScalars), hipMemcpyDeviceToHost, c.st));
  HIPCHECK(hipStreamSynchronize(c.st));
  if (c.sub_on) {
    // boundaries 0..5: transport, diffusion, reaction, second transport half, elasticity
    static const int slot[5] = {TUMOR_SUB_TRANSPORT, TUMOR_SUB_DIFFUSION, TUMOR_SUB_REACTION, TUMOR_SUB_TRANSPORT,
                                TUMOR_SUB_ELASTICITY};
    for (int k = 0; k < 5; ++k) {
      float ms = 0.f;
      HIPCHECK(hipEventElapsedTime(&ms, c.sub_ev[k], c.sub_ev[k + 1]));
      c.sub_ms[slot[k]] += ms;
    }
    c.sub_steps++;
  }
  bool any_bad = se.bad || c.hcs->bad;
  bool any_nc = !se.conv;
  for (int k = 0; k < 3; ++k) {
    any_bad |= sd[k].bad;
    any_nc |= !sd[k].conv;
  }
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    const double h = 2.0 * M_PI / c.n;
    for (int k = 0; k < 3; ++k) {
      stats->it_diff[k] = sd[k].it;
      stats->outer_diff[k] = sd[k].outer;
      stats->relres_diff[k] = sd[k].relres;
    }
    stats->it_elast = se.it;
    stats->outer_elast = se.outer;
    stats->relres_elast = se.relres;
    for (int k = 0; k < 8; ++k) stats->mass[k] = c.hcs->mass[k] * h * h * h;
    if (c.flags & TUMOR_F_ADVECTION) {
      const unsigned long long bits = c.hcs->cfl_bits;
      std::memcpy(&stats->max_cfl, &bits, sizeof(double));
      if (strang) stats->max_cfl *= 2.0;  // the half-steps measure |dt/2 v| / h
    } else {
      stats->max_cfl = 0.0;
    }
  }
  if (any_bad) {
    status = TUMOR_ENAN;
    g_err = "non-finite value or loss of positive definiteness in a solve";
  } else if (any_nc && status == TUMOR_OK) {
    status = TUMOR_ENOCONV;
    g_err = "a PCG solve reached max_it";
  }
}

// Physical <-> state transfers for the displacement (spectral in the state).
void u_to_phys(Ctx& c, const cplx<double>* U, double* dst) {
  for (int k = 0; k < 3; ++k) inv3<double>(c, U + k * c.S, dst + k * c.V, 1.0 / (double)c.V);
}
void u_from_phys(Ctx& c, const double* src, cplx<double>* U) {
  for (int k = 0; k < 3; ++k) fwd3<double>(c, src + k * c.V, nullptr, U + k * c.S);
}

template <typename R>
void apply_op_t(Ctx& c, int op, const double* in, double* out) {
  PrecBufs<R>& P = pb<R>(c);
  const long long V = c.V, S = c.S;
  const bool is64 = sizeof(R) == 8;
  // Spectral vectors for 3-component work: P.r (input spectra), P.q (outputs).
  cplx<R>* X = P.r;
  cplx<R>* Q = P.q;
  auto to_out = [&](const cplx<R>* spec, double* dst, double scale, int d) {
    if (is64) {
      inv3<R>(c, spec, reinterpret_cast<R*>(dst), scale, d);
    } else {
      R* tmp = reinterpret_cast<R*>(P.p);  // 3 S complex floats >= N^3 floats
      inv3<R>(c, spec, tmp, scale, d);
      tumor::launch_f32_to_f64(reinterpret_cast<const float*>(tmp), dst, V, c.st);
    }
  };
  tumor::KrylovArgs ka = kargs<R>(c, 1, X, c.sv64, 0.5 * c.cfg.dt, tumor::PREC_DIFF);
  switch (op) {
    case TUMOR_OP_DERIV_X:
    case TUMOR_OP_DERIV_Y:
    case TUMOR_OP_DERIV_Z:
      fwd3<R>(c, in, nullptr, X);
      to_out(X, out, 1.0 / (double)V, op - TUMOR_OP_DERIV_X);
      break;
    case TUMOR_OP_DIFFUSION:
      fwd3<R>(c, in, nullptr, X);
      diff_apply<R>(c, X, Q, 0.0, 1.0, nullptr);
      to_out(Q, out, 1.0 / (double)V, -1);
      break;
    case TUMOR_OP_CN_PRECOND:
      fwd3<R>(c, in, nullptr, X);
      tumor::launch_precond<R>(ka, X, Q, c.st);
      to_out(Q, out, 1.0 / (double)V, -1);
      break;
    case TUMOR_OP_ELASTICITY:
    case TUMOR_OP_ELAST_PRECOND:
      for (int k = 0; k < 3; ++k) fwd3<R>(c, in + k * V, nullptr, X + k * S);
      if (op == TUMOR_OP_ELASTICITY) {
        elast_apply<R>(c, X, Q, nullptr);
      } else {
        ka.ncomp = 3;
        ka.pc.kind = tumor::PREC_ELAST;
        tumor::launch_precond<R>(ka, X, Q, c.st);
      }
      for (int k = 0; k < 3; ++k) to_out(Q + k * S, out + k * V, 1.0 / (double)V, -1);
      break;
    default:
      throw Fail(TUMOR_EINVAL, "unknown operator id");
  }
}

// ------------------------------------------------------------------ adjoint
size_t slot_doubles(long long V) { return (size_t)(14 * V); }
size_t slot_bytes(long long V) { return (slot_doubles(V) * sizeof(double) + 255) & ~size_t(255); }

double* tape_slot(Ctx& c, int k) { return reinterpret_cast<double*>(c.tape + (size_t)k * slot_bytes(c.V)); }

// With a checkpoint every step (K = 1) the tape keeps every state X^0 .. X^T
// (T + 1 state slots) and, per step, the intermediates the transposes read:
// the transported p, i, n, g, w and the diffusion outputs i'', o', l'.  The
// reverse sweep then restores them instead of recomputing the step.
constexpr int kMidFields = 8;
size_t mid_bytes(long long V) { return ((size_t)kMidFields * V * sizeof(double) + 255) & ~size_t(255); }
double* mid_slot(Ctx& c, int m) {
  return reinterpret_cast<double*>(c.tape + (size_t)(c.rec_nsteps + 1) * slot_bytes(c.V) + (size_t)m * mid_bytes(c.V));
}
void save_mid(Ctx& c, double* slot) {
  enum { P, I, N, O, L, G, W, F };
  const size_t fb = c.V * sizeof(double);
  const double* src[kMidFields] = {c.G[P], c.G[I], c.G[N], c.G[G], c.G[W], c.Rdd[0], c.Rdd[1], c.Rdd[2]};
  for (int k = 0; k < kMidFields; ++k)
    HIPCHECK(hipMemcpyAsync(slot + k * c.V, src[k], fb, hipMemcpyDeviceToDevice, c.st));
}
void load_mid(Ctx& c, const double* slot) {
  enum { P, I, N, O, L, G, W, F };
  const size_t fb = c.V * sizeof(double);
  double* dst[kMidFields] = {c.G[P], c.G[I], c.G[N], c.G[G], c.G[W], c.Rdd[0], c.Rdd[1], c.Rdd[2]};
  for (int k = 0; k < kMidFields; ++k)
    HIPCHECK(hipMemcpyAsync(dst[k], slot + k * c.V, fb, hipMemcpyDeviceToDevice, c.st));
}
int n_ckpt(int nsteps, int K) { return (nsteps + K - 1) / K; }

void save_state(Ctx& c, double* slot) {
  const size_t fb = c.V * sizeof(double);
  for (int k = 0; k < 8; ++k) HIPCHECK(hipMemcpyAsync(slot + k * c.V, c.F[k], fb, hipMemcpyDeviceToDevice, c.st));
  const size_t ub = 3 * c.S * sizeof(cplx<double>);
  HIPCHECK(hipMemcpyAsync(slot + 8 * c.V, c.U, ub, hipMemcpyDeviceToDevice, c.st));
  HIPCHECK(hipMemcpyAsync(slot + 11 * c.V, c.Up, ub, hipMemcpyDeviceToDevice, c.st));
}

void load_state(Ctx& c, const double* slot) {
  const size_t fb = c.V * sizeof(double);
  for (int k = 0; k < 8; ++k) HIPCHECK(hipMemcpyAsync(c.F[k], slot + k * c.V, fb, hipMemcpyDeviceToDevice, c.st));
  const size_t ub = 3 * c.S * sizeof(cplx<double>);
  HIPCHECK(hipMemcpyAsync(c.U, slot + 8 * c.V, ub, hipMemcpyDeviceToDevice, c.st));
  HIPCHECK(hipMemcpyAsync(c.Up, slot + 11 * c.V, ub, hipMemcpyDeviceToDevice, c.st));
  refresh_state(c);
}

void zero(Ctx& c, double* p, long long count) {
  HIPCHECK(hipMemsetAsync(p, 0, count * sizeof(double), c.st));
}

// Adjoint solve A y = rhs (physical rhs, ncomp blocks) with x0 = 0; y stays
// spectral in c.Un.  kind: diffusion (A = 1 - dt/2 D_K) or elasticity.
SolveOut adjoint_solve(Ctx& c, int ncomp, const double* rhs, int which) {
  for (int k = 0; k < ncomp; ++k) fwd3<double>(c, rhs + k * c.V, nullptr, c.b64 + k * c.S);
  cplx<double>* x = c.Un;
  HIPCHECK(hipMemsetAsync(x, 0, ncomp * c.S * sizeof(cplx<double>), c.st));
  const double h = 0.5 * c.cfg.dt;
  auto r0 = [&](tumor::KrylovArgs& a) {
    a.ax = nullptr;
    tumor::launch_residual<double>(a, nullptr, c.st);
  };
  if (ncomp == 1) {
    auto A64 = [&](const cplx<double>* p, cplx<double>* q, const int* skip, const Fuse* fz = nullptr) {
      diff_apply<double>(c, p, q, 1.0, -h, skip, fz);
    };
    auto A32 = [&](const cplx<float>* p, cplx<float>* q, const int* skip, const Fuse* fz = nullptr) {
      diff_apply<float>(c, p, q, 1.0, -h, skip, fz);
    };
    return solve_system(c, 1, tumor::PREC_DIFF, h, x, c.b64, c.cfg.rtol_diff, which, A64, A32, r0);
  }
  auto A64 = [&](const cplx<double>* p, cplx<double>* q, const int* skip, const Fuse* fz = nullptr) {
    elast_apply<double>(c, p, q, skip, fz);
  };
  auto A32 = [&](const cplx<float>* p, cplx<float>* q, const int* skip, const Fuse* fz = nullptr) {
    elast_apply<float>(c, p, q, skip, fz);
  };
  return solve_system(c, 3, tumor::PREC_ELAST, 0.0, x, c.b64, c.cfg.rtol_elast, which, A64, A32, r0);
}

// CN adjoint of one field, given y = A^-1 cbar_plus (spectral): out = (1 + dt/2 D) y;
// KB += -dt/2 sum_a G_a y G_a (c- + c+).
void cn_adjoint_post(Ctx& c, const cplx<double>* y, double* out, const double* cm, const double* cp) {
  const double h = 0.5 * c.cfg.dt;
  PrecBufs<double>& P = c.p64;
  diff_apply<double>(c, y, P.q, 1.0, h, nullptr);
  inv3<double>(c, P.q, out, 1.0 / (double)c.V);
  fwd3<double>(c, cm, cp, P.r);  // spectrum of s = c- + c+
  // z and y inverse passes of y and s, then the three products on the x pass
  colp<double>(c, 2, true,
               Prog().in(0, y).in(1, P.r).out(P.A[0], {T1(0)}).out(P.A[1], {TW(0)}).out(P.A[2], {T1(1)}).out(
                   P.A[3], {TW(1)}));
  colp<double>(c, 1, true,
               Prog()
                   .in(0, P.A[0]).in(1, P.A[1]).in(2, P.A[2]).in(3, P.A[3])
                   .out(P.B[0], {T1(0)}).out(P.B[1], {TW(0)}).out(P.B[2], {T1(1)})
                   .out(P.B[3], {T1(2)}).out(P.B[4], {TW(2)}).out(P.B[5], {T1(3)}));
  const double iV = 1.0 / (double)c.V, cf = -h * iV * iV;
  DotProg d;
  for (int k = 0; k < 6; ++k) d.in(k, P.B[k]);
  d.out(c.KB, true)
      .prod(cf, fac({TW(0)}), fac({TW(3)}))
      .prod(cf, fac({T1(1)}), fac({T1(4)}))
      .prod(cf, fac({T1(2)}), fac({T1(5)}));
  tumor::launch_xdot<double>(c.n, d.a, P.tw, c.st);
}

// Coefficient sensitivities of the elasticity adjoint (Eqs. e:hook,
// e:variable_elasticity, e:screening) from y (spectral, in Un) and u (in U):
//   EB = -sum_a y_a u_a,  LB = -div y div u,  MB = -1/2 sum_ab S^y_ab S^u_ab,
// S_ab = G_b v_a + G_a v_b, and the physical y_a in Y[a].  The z and y inverse
// passes of each field leave eight partial transforms (v_x, v_y, v_z, dy v_x,
// dy v_y, dz v_x, dz v_z, dz v_y + dy v_z); one x pass forms every product.
void elast_sens(Ctx& c) {
  PrecBufs<double>& P = c.p64;
  const long long S = c.S;
  cplx<double>* const part[2][8] = {{P.B[0], P.B[1], P.B[2], P.B[3], P.B[4], P.B[5], P.B[6], P.B[7]},
                                     {P.r, P.r + S, P.r + 2 * S, P.p, P.p + S, P.p + 2 * S, P.q, P.q + S}};
  for (int f = 0; f < 2; ++f) {
    const cplx<double>* v = f == 0 ? c.Un : c.U;
    colp<double>(c, 2, true,
                 Prog()
                     .in(0, v).in(1, v + S).in(2, v + 2 * S)
                     .out(P.A[0], {T1(0)}).out(P.A[1], {T1(1)}).out(P.A[2], {T1(2)})
                     .out(P.A[3], {TW(0)}).out(P.A[4], {TW(2)}).out(P.A[5], {TW(1)}));
    cplx<double>* const* o = part[f];
    colp<double>(c, 1, true,
                 Prog()
                     .in(0, P.A[0]).in(1, P.A[1]).in(2, P.A[2]).in(3, P.A[3]).in(4, P.A[4]).in(5, P.A[5])
                     .out(o[0], {T1(0)}).out(o[1], {T1(1)}).out(o[2], {T1(2)})
                     .out(o[3], {TW(0)}).out(o[4], {TW(1)})
                     .out(o[5], {T1(3)}).out(o[6], {T1(4)}).out(o[7], {T1(5), TW(2)}));
  }
  DotProg d;
  for (int k = 0; k < 8; ++k) d.in(k, part[0][k]).in(8 + k, part[1][k]);
  // factors of the field whose partial transforms start at input b
  auto sxx = [](int b) { return fac({TW(b, 2.0)}); };
  auto syy = [](int b) { return fac({T1(b + 4, 2.0)}); };
  auto szz = [](int b) { return fac({T1(b + 6, 2.0)}); };
  auto sxy = [](int b) { return fac({T1(b + 3), TW(b + 1)}); };
  auto sxz = [](int b) { return fac({T1(b + 5), TW(b + 2)}); };
  auto syz = [](int b) { return fac({T1(b + 7)}); };
  auto dv = [](int b) { return fac({TW(b), T1(b + 4), T1(b + 6)}); };
  auto val = [](int b, int a) { return fac({T1(b + a)}); };
  const double iV = 1.0 / (double)c.V, iV2 = iV * iV;
  d.out(c.MB)
      .prod(-0.5 * iV2, sxx(0), sxx(8))
      .prod(-0.5 * iV2, syy(0), syy(8))
      .prod(-0.5 * iV2, szz(0), szz(8))
      .prod(-iV2, sxy(0), sxy(8))
      .prod(-iV2, sxz(0), sxz(8))
      .prod(-iV2, syz(0), syz(8));
  d.out(c.LB).prod(-iV2, dv(0), dv(8));
  d.out(c.EB).prod(-iV2, val(0, 0), val(8, 0)).prod(-iV2, val(0, 1), val(8, 1)).prod(-iV2, val(0, 2), val(8, 2));
  for (int a = 0; a < 3; ++a) d.out(c.Y[a]).prod(iV, val(0, a));
  tumor::launch_xdot<double>(c.n, d.a, P.tw, c.st);
}

// Adjoint of the force b = zeta tanh(tau) G tau, tau = p' + n' (Eq. e:force),
// with b_bar = -y: TB = sum_a [-zeta sech^2(tau) G_a tau y_a] - div W,
// W_a = -zeta tanh(tau) y_a.  G tau comes from one inverse transform with three
// outputs; div W from one forward transform that sums the three derivatives
// and one inverse transform.
void force_adj(Ctx& c) {
  PrecBufs<double>& P = c.p64;
  const long long V = c.V;
  const double iV = 1.0 / (double)V;
  enum { kP = 0, kN = 2 };  // p and n in F
  fwd3<double>(c, c.F[kP], c.F[kN], P.r);  // spectrum of tau
  colp<double>(c, 2, true, Prog().in(0, P.r).out(P.A[0], {T1(0)}).out(P.A[1], {TW(0)}));
  colp<double>(c, 1, true, Prog().in(0, P.A[0]).in(1, P.A[1]).out(P.B[0], {T1(0)}).out(P.B[1], {TW(0)}).out(
                               P.B[2], {T1(1)}));
  Prog gx;
  gx.in(0, P.B[0]).in(1, P.B[1]).in(2, P.B[2]).out(c.T[0], {TW(0)}).out(c.T[1], {T1(1)}).out(c.T[2], {T1(2)});
  tumor::launch_xinv<double>(c.n, to_x(gx.p, iV), P.tw, c.st);
  zero(c, c.TB, V);
  // pointwise part; W_a replaces G_a tau in T[a]
  for (int a = 0; a < 3; ++a)
    tumor::launch_force_adj(V, c.prm.zeta, c.F[kP], c.F[kN], c.T[a], c.Y[a], c.TB, c.T[a], c.st);
  Prog fx;
  fx.in(0, c.T[0]).in(1, c.T[1]).in(2, c.T[2]).out(P.A[0], {T1(0)}).out(P.A[1], {T1(1)}).out(P.A[2], {T1(2)});
  tumor::launch_xfwd<double>(c.n, to_x(fx.p, 1.0), P.tw, c.st, true);
  // spectra of W_x and of dy W_y + dz W_z (the x derivative of W_x waits for the inverse x pass)
  colp<double>(c, 1, false,
               Prog().in(0, P.A[0]).in(1, P.A[1]).in(2, P.A[2]).out(P.B[0], {T1(0)}).out(P.B[1], {TW(1)}).out(
                   P.B[2], {T1(2)}));
  colp<double>(c, 2, false, Prog().in(0, P.B[0]).in(1, P.B[1]).in(2, P.B[2]).out(P.A[0], {T1(0)}).out(
                                P.A[1], {T1(1), TW(2)}));
  colp<double>(c, 2, true, Prog().in(0, P.A[0]).in(1, P.A[1]).out(P.B[0], {T1(0)}).out(P.B[1], {T1(1)}));
  colp<double>(c, 1, true, Prog().in(0, P.B[0]).in(1, P.B[1]).out(P.A[0], {T1(0)}).out(P.A[1], {T1(1)}));
  Prog dx;
  dx.in(0, P.A[0]).in(1, P.A[1]).out(c.T[3], {TW(0), T1(1)});
  tumor::launch_xinv<double>(c.n, to_x(dx.p, iV), P.tw, c.st);
  tumor::launch_axpy(V, -1.0, c.T[3], c.TB, c.st);
}

// Reverse one recorded step.  On entry the forward step from X^m has just been
// recomputed: F = q^{m+1}, U = u^{m+1}, Up = u^m, G = transported fields,
// Rdd = (i'', o', l'), vel = (v^m, div v^m); x0 holds X^m.
void adjoint_core(Ctx& c, const double* x0, double* adj, int m, double* grad) {
  enum { P, I, N, O, L, G, W, F };
  const long long V = c.V;
  double* Lm[14];
  for (int k = 0; k < 14; ++k) Lm[k] = adj + k * V;
  const double* F0[8];
  for (int k = 0; k < 8; ++k) F0[k] = x0 + k * V;
  const double iV = 1.0 / (double)V;
  HIPCHECK(hipMemsetAsync(c.gs, 0, sizeof(tumor::GradScalars), c.st));
  zero(c, c.KB, V);
  PrecBufs<double>& PB = c.p64;
  // ---- S6 elasticity and force, S5 mixture
  if (c.flags & TUMOR_F_ELASTICITY) {
    adjoint_solve(c, 3, Lm[8], 7);  // y (spectral) in Un
    elast_sens(c);
    force_adj(c);
    tumor::launch_axpy(V, 1.0, c.TB, Lm[P], c.st);
    tumor::launch_axpy(V, 1.0, c.TB, Lm[N], c.st);
    tumor::CoefAdjArgs ca;
    std::memset(&ca, 0, sizeof(ca));
    ca.mub = c.MB;
    ca.lamb = c.LB;
    ca.etab = c.EB;
    ca.p1 = c.F[P];
    ca.i1 = c.F[I];
    ca.n1 = c.F[N];
    ca.g1 = c.F[G];
    ca.w1 = c.F[W];
    ca.f1 = c.F[F];
    ca.bg = c.BG;
    for (int k = 0; k < 8; ++k) ca.L[k] = Lm[k];
    ca.fc = c.fc;
    ca.inv_scale = 1.0 / c.prm.lame_scale;
    ca.partials = c.partials;
    ca.gs = c.gs;
    ca.V = V;
    tumor::launch_coef_adj(ca, c.st);
  } else {
    for (int a = 0; a < 3; ++a) tumor::launch_axpy(V, 1.0, Lm[8 + a], Lm[11 + a], c.st);
  }
  // ---- S4b, S4, S3
  {
    tumor::ReactAdjArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.p_dag = c.G[P];
    ra.i_dag = c.G[I];
    ra.i_dd = c.Rdd[0];
    ra.g_dag = c.G[G];
    ra.w_dag = c.G[W];
    ra.o_dag = c.Rdd[1];
    ra.i1 = c.F[I];
    ra.g1 = c.F[G];
    ra.w1 = c.F[W];
    ra.w0 = F0[W];
    ra.g0 = F0[G];
    ra.rho_w = c.prm.rho_w;
    ra.rho_g = c.prm.rho_g;
    const int ids[7] = {P, I, N, O, L, G, W};
    for (int k = 0; k < 7; ++k) ra.L[k] = Lm[ids[k]];
    ra.idd = c.IDD;
    ra.ddb = c.DDB;
    ra.rb = c.RB;
    ra.V = V;
    ra.rc = c.rc;
    tumor::launch_react_adj(ra, c.st);
  }
  // ---- S2 (coefficients K of the step start)
  {
    const double* in[9] = {F0[P], F0[I], F0[I], F0[N], F0[G], F0[W], F0[O], F0[L], F0[F]};
    double* out[8] = {nullptr};
    refresh(c, 0, in, out);
  }
  {
    // the three (two without edema) adjoint CN solves as one batched solve
    const int ns = (c.flags & TUMOR_F_EDEMA) ? 3 : 2;
    const double* rhs[3] = {c.IDD, Lm[O], Lm[L]};
    const int which[3] = {4, 5, 6};
    SolveOut so[3];
    cn_solve_b(c, ns, rhs, nullptr, which, so, true);
    double* const out[3] = {Lm[I], Lm[O], Lm[L]};
    const double* const cm[3] = {c.G[I], F0[O], F0[L]};
    const double* const cp[3] = {c.Rdd[0], c.Rdd[1], c.Rdd[2]};
    for (int k = 0; k < ns; ++k) cn_adjoint_post(c, c.Un + k * c.S, out[k], cm[k], cp[k]);
  }
  tumor::launch_axpy(V, -1.0, c.DDB, Lm[I], c.st);
  // ---- S1 transport
  if (c.flags & TUMOR_F_ADVECTION) {
    for (int k = 0; k < 6; ++k) zero(c, c.SLO[k], V);
    zero(c, c.DB, V);
    for (int k = 0; k < 3; ++k) zero(c, c.VB[k], V);
    tumor::SLAdjArgs sa;
    sa.vx = c.vel[0];
    sa.vy = c.vel[1];
    sa.vz = c.vel[2];
    sa.div = c.vel[3];
    const int ids[6] = {P, I, N, G, W, F};
    for (int k = 0; k < 6; ++k) {
      sa.q[k] = F0[ids[k]];
      sa.lam[k] = Lm[ids[k]];
      sa.out[k] = c.SLO[k];
    }
    sa.divb = c.DB;
    for (int k = 0; k < 3; ++k) sa.vb[k] = c.VB[k];
    sa.n_grid = c.n;
    sa.dt = c.cfg.dt;
    sa.s = c.cfg.dt / (2.0 * M_PI / c.n);
    tumor::launch_sl_adj(sa, c.gs, c.st);
    fwd3<double>(c, c.DB, nullptr, PB.r);
    for (int a = 0; a < 3; ++a) {
      inv3<double>(c, PB.r, c.T[0], iV, a);
      tumor::launch_axpy(V, -1.0, c.T[0], c.VB[a], c.st);
    }
    for (int k = 0; k < 6; ++k)
      HIPCHECK(hipMemcpyAsync(Lm[ids[k]], c.SLO[k], V * sizeof(double), hipMemcpyDeviceToDevice, c.st));
  } else {
    for (int k = 0; k < 3; ++k) zero(c, c.VB[k], V);
  }
  // ---- S0
  {
    tumor::S0AdjArgs sa;
    sa.Kb = c.KB;
    sa.rb = c.RB;
    sa.w0 = F0[W];
    sa.g0 = F0[G];
    sa.f0 = F0[F];
    sa.Lw = Lm[W];
    sa.Lg = Lm[G];
    sa.Lf = Lm[F];
    sa.k_w = c.prm.k_w;
    sa.k_g = c.prm.k_g;
    sa.k_f = c.prm.k_f;
    sa.rho_w = c.prm.rho_w;
    sa.rho_g = c.prm.rho_g;
    sa.partials = c.partials;
    sa.gs = c.gs;
    sa.V = V;
    tumor::launch_s0_adj(sa, c.st);
  }
  // ---- displacement slots: v = (u^m - u^{m-1}) / dt
  const double idt = 1.0 / c.cfg.dt;
  for (int a = 0; a < 3; ++a) {
    tumor::launch_xpay(V, Lm[11 + a], idt, c.VB[a], Lm[8 + a], c.st);
    HIPCHECK(hipMemsetAsync(Lm[11 + a], 0, V * sizeof(double), c.st));
    tumor::launch_axpy(V, -idt, c.VB[a], Lm[11 + a], c.st);
  }
  // ---- initial-condition weights after the first step
  double* icg = nullptr;
  if (m == 0 && c.n_ic > 0) {
    HIPCHECK(hipMemcpyAsync(c.T[2], c.ic_host, 5 * (size_t)c.n_ic * sizeof(double), hipMemcpyHostToDevice, c.st));
    tumor::launch_ic_adj(c.n, c.T[2], c.n_ic, Lm[P], c.T[3], c.T[1], c.st);
    icg = c.T[1];
  }
  HIPCHECK(hipGetLastError());
  tumor::GradScalars hg;
  HIPCHECK(hipMemcpyAsync(&hg, c.gs, sizeof(hg), hipMemcpyDeviceToHost, c.st));
  std::vector<double> gic(c.n_ic > 0 ? c.n_ic : 1);
  if (icg) HIPCHECK(hipMemcpyAsync(gic.data(), icg, c.n_ic * sizeof(double), hipMemcpyDeviceToHost, c.st));
  HIPCHECK(hipStreamSynchronize(c.st));
  for (int k = 0; k < 5; ++k) grad[k] += hg.g[k];
  if (icg)
    for (int k = 0; k < c.n_ic; ++k) grad[5 + k] += gic[k];
}

template <typename Fn>
int guarded(Fn fn) {
  try {
    return fn();
  } catch (const Fail& f) {
    g_err = f.what();
    return f.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return TUMOR_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return TUMOR_EDEVICE;
  }
}

int einval(const char* msg) {
  g_err = msg;
  return TUMOR_EINVAL;
}

}  // namespace

// ===================================================================== C ABI
extern "C" {

int tumor_abi_version(void) { return TUMOR_ABI_VERSION; }

const char* tumor_last_error(void) { return g_err.c_str(); }

int tumor_workspace_bytes(const tumor_config* cfg, size_t* bytes) {
  if (!bytes) return einval("bytes is NULL");
  if (check_cfg(cfg) != TUMOR_OK) return einval("invalid tumor_config");
  *bytes = workspace_size(*cfg);
  return TUMOR_OK;
}

}  // extern "C"

// ------------------------------------------------ allocation-free contexts
// One fixed workspace per GPU for tumor_init_static, in device memory that the
// code object itself reserves (held until the process ends).  In host code its
// name is only a stand-in: the device address comes from hipGetSymbolAddress,
// once per device, and only that address is ever passed on.
static __device__ __align__(256) unsigned char scratch[TUMOR_STATIC_WS_BYTES];

namespace {

// Argument checks shared by tumor_init and tumor_init_static.
int check_init(const tumor_config* cfg, const tumor_params* prm, const double* wm, const double* gm,
               const double* csf, int32_t n_ic, const double* ic_centers, const double* ic_sigmas,
               const double* ic_weights) {
  if (check_cfg(cfg) != TUMOR_OK) return einval("invalid tumor_config");
  if (check_params(prm) != TUMOR_OK) return einval("invalid tumor_params");
  if (!wm || !gm || !csf) return einval("tissue map pointer is NULL");
  if (n_ic < 0) return einval("n_ic < 0");
  if (n_ic > 0 && (!ic_centers || !ic_sigmas || !ic_weights)) return einval("initial-condition array is NULL");
  for (int k = 0; k < n_ic; ++k) {
    if (!(ic_sigmas[k] > 0.0) || !std::isfinite(ic_sigmas[k])) return einval("ic_sigmas must be > 0");
    if (!std::isfinite(ic_weights[k])) return einval("ic_weights must be finite");
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(ic_centers[3 * k + a])) return einval("ic_centers must be finite");
  }
  const long long V = (long long)cfg->n * cfg->n * cfg->n;
  if (5LL * n_ic > V) return einval("too many initial-condition centres for this grid");
  return TUMOR_OK;
}

// Set up a context whose host storage (c itself, c->hsv, c->hcs and c->ic_host
// with room for 5 n_ic + 1 doubles) the caller provides, on `workspace`.
// Allocates nothing: device work is copies, fills and kernels.
int init_context(Ctx* c, const tumor_config* cfg, const tumor_params* prm, void* workspace, const double* wm,
                 const double* gm, const double* csf, int32_t n_ic, const double* ic_centers,
                 const double* ic_sigmas, const double* ic_weights, void* hip_stream) {
  return guarded([&]() -> int {
    const long long V = (long long)cfg->n * cfg->n * cfg->n;
    c->cfg = *cfg;
    c->prm = *prm;
    c->st = static_cast<hipStream_t>(hip_stream);
    c->n = cfg->n;
    c->V = V;
    c->S = V / 2;
    c->mixed = cfg->precision == TUMOR_PREC_MIXED;
    c->single = cfg->model == TUMOR_MODEL_SINGLE;
    c->adj = (cfg->flags & TUMOR_F_ADJOINT) != 0;
    c->flags = ((cfg->flags & TUMOR_F_DEFAULT) == 0 ? TUMOR_F_DEFAULT : (cfg->flags & TUMOR_F_DEFAULT)) |
               (cfg->flags & TUMOR_F_STRANG);
    c->win_start = -1;
    int dev_count = 0;
    if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1) throw Fail(TUMOR_EDEVICE, "no HIP device");
    Carver cv{static_cast<char*>(workspace), 0, false};
    layout(*c, cv);
    c->pred[0] = c->pred[1] = c->pred[2] = c->pred[4] = c->pred[5] = c->pred[6] = 6;
    c->pred[3] = c->pred[7] = 30;
    for (int w = 0; w < 8; ++w) {
      c->pred_in[w][0] = c->pred[w] * 2 / 3;
      c->pred_in[w][1] = c->pred_in[w][2] = std::max(1, c->pred[w] / 3);
    }
    c->cur_tag = -1;
    set_consts(*c);
    twiddles(*c);
    HIPCHECK(hipMemsetAsync(c->sv64, 0, tumor::kMaxSys * sizeof(tumor::SolveScalars), c->st));
    HIPCHECK(hipMemsetAsync(c->sv32, 0, tumor::kMaxSys * sizeof(tumor::SolveScalars), c->st));
    HIPCHECK(hipMemsetAsync(c->cs, 0, sizeof(tumor::CoefScalars), c->st));
    enum { P, I, N, O, L, G, W, F };
    const size_t fb = V * sizeof(double);
    HIPCHECK(hipMemcpyAsync(c->F[G], gm, fb, hipMemcpyDeviceToDevice, c->st));
    HIPCHECK(hipMemcpyAsync(c->F[W], wm, fb, hipMemcpyDeviceToDevice, c->st));
    HIPCHECK(hipMemcpyAsync(c->F[F], csf, fb, hipMemcpyDeviceToDevice, c->st));
    HIPCHECK(hipMemsetAsync(c->F[I], 0, fb, c->st));
    HIPCHECK(hipMemsetAsync(c->F[N], 0, fb, c->st));
    HIPCHECK(hipMemsetAsync(c->F[L], 0, fb, c->st));
    HIPCHECK(hipMemsetAsync(c->BG, 0, fb, c->st));
    tumor::launch_fill(c->F[O], prm->o_heal, V, c->st);
    double* ic = c->ic_host;
    for (int k = 0; k < n_ic; ++k) {
      ic[5 * k + 0] = ic_centers[3 * k + 0];
      ic[5 * k + 1] = ic_centers[3 * k + 1];
      ic[5 * k + 2] = ic_centers[3 * k + 2];
      ic[5 * k + 3] = ic_sigmas[k];
      ic[5 * k + 4] = ic_weights[k];
    }
    if (n_ic > 0)
      HIPCHECK(hipMemcpyAsync(c->G[0], ic, 5 * (size_t)n_ic * sizeof(double), hipMemcpyHostToDevice, c->st));
    tumor::launch_ic(c->n, c->G[0], n_ic, c->F[P], c->st);
    c->n_ic = n_ic;
    const size_t ub = 3 * c->S * sizeof(cplx<double>);
    HIPCHECK(hipMemsetAsync(c->U, 0, ub, c->st));
    HIPCHECK(hipMemsetAsync(c->Up, 0, ub, c->st));
    HIPCHECK(hipMemsetAsync(c->Un, 0, ub, c->st));
    refresh_state(*c);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(c->st));
    return TUMOR_OK;
  });
}

constexpr int kStaticDevices = 64;
constexpr int kStaticMaxIC = 256;

struct StaticSlot {
  void* ws;      // device address of `scratch` on this device (null until looked up)
  bool in_use;   // a live context holds the array
  tumor_ctx ctx;
  tumor::SolveScalars hsv[tumor::kMaxSys];
  tumor::CoefScalars hcs;
  double ic[5 * kStaticMaxIC + 1];
};
StaticSlot g_static[kStaticDevices];
std::mutex g_static_mu;

}  // namespace

extern "C" {

int tumor_init(tumor_ctx** out, const tumor_config* cfg, const tumor_params* prm, void* workspace,
               size_t ws_bytes, const double* wm, const double* gm, const double* csf, int32_t n_ic,
               const double* ic_centers, const double* ic_sigmas, const double* ic_weights, void* hip_stream) {
  if (!out) return einval("out is NULL");
  *out = nullptr;
  int rc = check_init(cfg, prm, wm, gm, csf, n_ic, ic_centers, ic_sigmas, ic_weights);
  if (rc != TUMOR_OK) return rc;
  if (!workspace) return einval("workspace is NULL");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return einval("workspace is not 256-byte aligned");
  const size_t need = workspace_size(*cfg);
  if (ws_bytes < need) {
    g_err = "workspace too small: need " + std::to_string(need) + " bytes";
    return TUMOR_ENOMEM;
  }
  tumor_ctx* c = new (std::nothrow) tumor_ctx;
  if (!c) {
    g_err = "host allocation failed";
    return TUMOR_ENOMEM;
  }
  std::memset(c, 0, sizeof(*c));
  c->static_dev = -1;
  c->ic_host = new (std::nothrow) double[5 * (size_t)n_ic + 1];
  void* h1 = nullptr;
  void* h2 = nullptr;
  if (c->ic_host && hipHostMalloc(&h1, tumor::kMaxSys * sizeof(tumor::SolveScalars), hipHostMallocDefault) == hipSuccess &&
      hipHostMalloc(&h2, sizeof(tumor::CoefScalars), hipHostMallocDefault) == hipSuccess) {
    c->hsv = static_cast<tumor::SolveScalars*>(h1);
    c->hcs = static_cast<tumor::CoefScalars*>(h2);
    rc = init_context(c, cfg, prm, workspace, wm, gm, csf, n_ic, ic_centers, ic_sigmas, ic_weights, hip_stream);
  } else {
    g_err = "host allocation failed";
    rc = TUMOR_ENOMEM;
  }
  if (rc != TUMOR_OK) {
    if (h1) (void)hipHostFree(h1);
    if (h2) (void)hipHostFree(h2);
    delete[] c->ic_host;
    delete c;
    return rc;
  }
  *out = c;
  return TUMOR_OK;
}

int tumor_init_static(tumor_ctx** out, const tumor_config* cfg, const tumor_params* prm, const double* wm,
                      const double* gm, const double* csf, int32_t n_ic, const double* ic_centers,
                      const double* ic_sigmas, const double* ic_weights, void* hip_stream) {
  if (!out) return einval("out is NULL");
  *out = nullptr;
  int rc = check_init(cfg, prm, wm, gm, csf, n_ic, ic_centers, ic_sigmas, ic_weights);
  if (rc != TUMOR_OK) return rc;
  const size_t need = workspace_size(*cfg);
  if (need > (size_t)TUMOR_STATIC_WS_BYTES) {
    g_err = "configuration needs " + std::to_string(need) + " bytes of workspace; the allocation-free context holds " +
            std::to_string((size_t)TUMOR_STATIC_WS_BYTES) + " (n <= 32)";
    return TUMOR_EINVAL;
  }
  if (n_ic > kStaticMaxIC) return einval("the allocation-free context holds at most 256 initial-condition centres");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
    g_err = "no current HIP device";
    return TUMOR_EDEVICE;
  }
  if (dev >= kStaticDevices) return einval("device index beyond the allocation-free context table");
  std::lock_guard<std::mutex> lock(g_static_mu);
  StaticSlot& s = g_static[dev];
  if (s.in_use) {
    g_err = "the allocation-free workspace of this device is held by a live context";
    return TUMOR_ESTATE;
  }
  if (!s.ws) {
    // once per device, with that device current (hipGetDevice above)
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      g_err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
      return TUMOR_EDEVICE;
    }
    s.ws = ptr;
  }
  tumor_ctx* c = &s.ctx;
  std::memset(c, 0, sizeof(*c));
  c->static_dev = dev;
  c->hsv = s.hsv;
  c->hcs = &s.hcs;
  c->ic_host = s.ic;
  rc = init_context(c, cfg, prm, s.ws, wm, gm, csf, n_ic, ic_centers, ic_sigmas, ic_weights, hip_stream);
  if (rc != TUMOR_OK) return rc;
  s.in_use = true;
  *out = c;
  return TUMOR_OK;
}

int tumor_step(tumor_ctx* ctx, int32_t nsteps, tumor_step_stats* last) {
  if (!ctx) return einval("ctx is NULL");
  if (nsteps < 0) return einval("nsteps < 0");
  return guarded([&]() -> int {
    int status = TUMOR_OK;
    tumor_step_stats st;
    Ctx& c = *ctx;
    for (int s = 0; s < nsteps; ++s) {
      int m = -1;  // index of the step being recorded
      if (c.rec_active && c.rev_done == 0 && c.rec_steps < c.rec_nsteps) {
        if (c.rec_steps % c.rec_K == 0) save_state(c, tape_slot(c, c.rec_steps / c.rec_K));
        m = c.rec_steps++;
      }
      do_step(c, &st, status);
      if (status == TUMOR_ENAN) break;
      if (m >= 0 && c.rec_K == 1) {
        save_mid(c, mid_slot(c, m));
        if (m == c.rec_nsteps - 1) save_state(c, tape_slot(c, c.rec_nsteps));
      }
    }
    if (last && nsteps > 0) *last = st;
    return status;
  });
}

int tumor_solve_elasticity(tumor_ctx* ctx, const double* force, double* u_out, int32_t* iters, double* relres) {
  if (!ctx) return einval("ctx is NULL");
  if (!u_out) return einval("u_out is NULL");
  return guarded([&]() -> int {
    Ctx& c = *ctx;
    enum { P, I, N };
    if (force) {
      for (int k = 0; k < 3; ++k) fwd3<double>(c, force + k * c.V, nullptr, c.b64 + k * c.S, -1.0);
    } else {
      force_rhs(c, c.F[P], c.F[N], c.b64);
    }
    SolveOut so = elast_solve(c, c.Un, -1);
    u_to_phys(c, c.Un, u_out);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(c.st));
    if (iters) *iters = so.it;
    if (relres) *relres = so.relres;
    if (so.bad) {
      g_err = "non-finite value in the elasticity solve";
      return TUMOR_ENAN;
    }
    if (!so.conv) {
      g_err = "elasticity PCG reached max_it";
      return TUMOR_ENOCONV;
    }
    return TUMOR_OK;
  });
}

int tumor_transport(tumor_ctx* ctx, double* out, double* max_cfl) {
  if (!ctx) return einval("ctx is NULL");
  if (!out) return einval("out is NULL");
  return guarded([&]() -> int {
    Ctx& c = *ctx;
    enum { P, I, N, O, L, G, W, F };
    const double* const ins[6] = {c.F[P], c.F[I], c.F[N], c.F[G], c.F[W], c.F[F]};
    double* const outs[6] = {out, out + c.V, out + 2 * c.V, out + 3 * c.V, out + 4 * c.V, out + 5 * c.V};
    transport(c, ins, outs);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(c.hcs, c.cs, sizeof(tumor::CoefScalars), hipMemcpyDeviceToHost, c.st));
    HIPCHECK(hipStreamSynchronize(c.st));
    if (max_cfl) {
      const unsigned long long bits = c.hcs->cfl_bits;
      std::memcpy(max_cfl, &bits, sizeof(double));
    }
    return TUMOR_OK;
  });
}

int tumor_diagnose(tumor_ctx* ctx, double threshold, double* fields, tumor_diagnostics* out) {
  if (!ctx) return einval("ctx is NULL");
  if (!out) return einval("out is NULL");
  if (!(threshold >= 0.0) || !std::isfinite(threshold)) return einval("threshold must be finite and >= 0");
  return guarded([&]() -> int {
    Ctx& c = *ctx;
    PrecBufs<double>& P = c.p64;
    auto** A = P.A;
    auto** B = P.B;
    const long long S = c.S;
    // u_a and F_ab = G_b u_a in physical space (FP64 in both precisions).
    // Scratch: the pass buffers, the post-transport species G and the velocity
    // buffers, none of which carries state between calls.
    colp<double>(c, 2, true,
                 Prog()
                     .in(0, c.U)
                     .in(1, c.U + S)
                     .in(2, c.U + 2 * S)
                     .out(A[0], {T1(0)})
                     .out(A[1], {T1(1)})
                     .out(A[2], {T1(2)})
                     .out(A[3], {TW(0)})
                     .out(A[4], {TW(1)})
                     .out(A[5], {TW(2)}));
    colp<double>(c, 1, true,
                 Prog()
                     .in(0, A[0])
                     .in(1, A[1])
                     .in(2, A[2])
                     .in(3, A[3])
                     .in(4, A[4])
                     .out(B[0], {T1(0)})
                     .out(B[1], {T1(1)})
                     .out(B[2], {T1(2)})
                     .out(B[3], {TW(0)})
                     .out(B[4], {TW(1)})
                     .out(B[5], {TW(2)})
                     .out(B[6], {T1(3)})
                     .out(B[7], {T1(4)}));
    colp<double>(c, 1, true, Prog().in(0, A[5]).out(A[0], {T1(0)}));
    double* ph[12] = {c.G[0], c.G[1], c.G[2], c.G[3], c.G[4], c.G[5], c.G[6], c.G[7],
                      c.vel[0], c.vel[1], c.vel[2], c.vel[3]};
    Prog x1;
    for (int k = 0; k < 6; ++k) x1.in(k, B[k]);
    x1.out(ph[0], {T1(0)}).out(ph[1], {T1(1)}).out(ph[2], {T1(2)});
    x1.out(ph[3], {TW(0)}).out(ph[4], {TW(1)}).out(ph[5], {TW(2)});
    x1.out(ph[6], {T1(3)}).out(ph[7], {T1(4)});
    Prog x2;
    x2.in(0, B[5]).in(1, B[6]).in(2, B[7]).in(3, A[0]);
    x2.out(ph[8], {T1(0)}).out(ph[9], {T1(1)}).out(ph[10], {T1(2)}).out(ph[11], {T1(3)});
    const double inv = 1.0 / (double)c.V;
    tumor::launch_xinv<double>(c.n, to_x(x1.p, inv), P.tw, c.st);
    tumor::launch_xinv<double>(c.n, to_x(x2.p, inv), P.tw, c.st);
    tumor::DiagArgs d;
    std::memset(&d, 0, sizeof(d));
    for (int k = 0; k < 12; ++k) d.f[k] = ph[k];
    d.mu = c.mu;
    d.lam = c.lam;
    double* icd = reinterpret_cast<double*>(A[6]);
    double* res = reinterpret_cast<double*>(A[7]);
    if (c.n_ic > 0)
      HIPCHECK(hipMemcpyAsync(icd, c.ic_host, 5 * (size_t)c.n_ic * sizeof(double), hipMemcpyHostToDevice, c.st));
    d.ic = icd;
    d.n_ic = c.n_ic;
    d.n = c.n;
    d.h = 2.0 * M_PI / c.n;
    d.thr = threshold;
    if (fields) {
      d.trace = fields;
      d.shear = fields + c.V;
      d.jac = fields + 2 * c.V;
    }
    d.partials = c.partials;
    tumor::launch_diag(d, res, c.st);
    HIPCHECK(hipGetLastError());
    double r[8];
    HIPCHECK(hipMemcpyAsync(r, res, sizeof(r), hipMemcpyDeviceToHost, c.st));
    HIPCHECK(hipStreamSynchronize(c.st));
    out->max_disp = r[0];
    out->trace_min = r[1];
    out->trace_max = r[2];
    out->shear_max = r[3];
    out->jac_min = r[4];
    out->jac_max = r[5];
    out->jac_l2 = r[6];
    out->d_max = r[7];
    return TUMOR_OK;
  });
}

int tumor_get_field(tumor_ctx* ctx, int32_t id, double* dst) {
  if (!ctx) return einval("ctx is NULL");
  if (!dst) return einval("dst is NULL");
  if (id < 0 || id >= TUMOR_FIELD_COUNT) return einval("unknown field id");
  return guarded([&]() -> int {
    Ctx& c = *ctx;
    const size_t fb = c.V * sizeof(double);
    if (id < 8) {
      HIPCHECK(hipMemcpyAsync(dst, c.F[id], fb, hipMemcpyDeviceToDevice, c.st));
    } else if (id == TUMOR_FIELD_U || id == TUMOR_FIELD_UPREV) {
      u_to_phys(c, id == TUMOR_FIELD_U ? c.U : c.Up, dst);
    } else {
      const double* src[6] = {c.K, c.rho, c.mu, c.lam, c.eta, c.BG};
      HIPCHECK(hipMemcpyAsync(dst, src[id - TUMOR_FIELD_K], fb, hipMemcpyDeviceToDevice, c.st));
    }
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(c.st));
    return TUMOR_OK;
  });
}

int tumor_set_field(tumor_ctx* ctx, int32_t id, const double* src) {
  if (!ctx) return einval("ctx is NULL");
  if (!src) return einval("src is NULL");
  if (id < 0 || (id > TUMOR_FIELD_UPREV && id != TUMOR_FIELD_BG)) return einval("field is not settable");
  return guarded([&]() -> int {
    Ctx& c = *ctx;
    if (id < 8) {
      HIPCHECK(hipMemcpyAsync(c.F[id], src, c.V * sizeof(double), hipMemcpyDeviceToDevice, c.st));
    } else if (id == TUMOR_FIELD_BG) {
      HIPCHECK(hipMemcpyAsync(c.BG, src, c.V * sizeof(double), hipMemcpyDeviceToDevice, c.st));
    } else {
      u_from_phys(c, src, id == TUMOR_FIELD_U ? c.U : c.Up);
    }
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(c.st));
    return TUMOR_OK;
  });
}

int tumor_refresh(tumor_ctx* ctx) {
  if (!ctx) return einval("ctx is NULL");
  return guarded([&]() -> int {
    refresh_state(*ctx);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(ctx->st));
    return TUMOR_OK;
  });
}

int tumor_apply_op(tumor_ctx* ctx, int32_t op, const double* in, double* out) {
  if (!ctx) return einval("ctx is NULL");
  if (!in || !out) return einval("in/out is NULL");
  if (op < 0 || op >= TUMOR_OP_COUNT) return einval("unknown operator id");
  return guarded([&]() -> int {
    Ctx& c = *ctx;
    if (op == TUMOR_OP_FORCE) {
      force_rhs(c, in, nullptr, c.b64);
      for (int k = 0; k < 3; ++k) inv3<double>(c, c.b64 + k * c.S, out + k * c.V, -1.0 / (double)c.V);
    } else if (c.mixed) {
      apply_op_t<float>(c, op, in, out);
    } else {
      apply_op_t<double>(c, op, in, out);
    }
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(c.st));
    return TUMOR_OK;
  });
}

int tumor_interp(tumor_ctx* ctx, const double* q, const double* jx, const double* jy, const double* jz,
                 int64_t count, double* out) {
  if (!ctx) return einval("ctx is NULL");
  if (count < 0 || count > (int64_t(1) << 40)) return einval("count out of range");
  if (count > 0 && (!q || !jx || !jy || !jz || !out)) return einval("NULL array");
  return guarded([&]() -> int {
    tumor::launch_interp(ctx->n, q, jx, jy, jz, count, out, ctx->st);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(ctx->st));
    return TUMOR_OK;
  });
}

int tumor_force_iterations(tumor_ctx* ctx, const int32_t* iters) {
  if (!ctx) return einval("ctx is NULL");
  if (!iters) {
    ctx->has_forced = false;
    return TUMOR_OK;
  }
  if (ctx->mixed) return einval("forced iteration counts apply to the FP64 precision only");
  for (int k = 0; k < 4; ++k) {
    if (iters[k] < -1 || iters[k] > ctx->cfg.max_it) return einval("forced count out of range");
    ctx->forced[k] = iters[k];
  }
  ctx->has_forced = true;
  return TUMOR_OK;
}

int tumor_tape_bytes(const tumor_config* cfg, int32_t nsteps, int32_t ckpt_every, size_t* bytes) {
  if (check_cfg(cfg) != TUMOR_OK) return einval("invalid tumor_config");
  if (!bytes) return einval("bytes is NULL");
  if (nsteps < 1 || ckpt_every < 1) return einval("nsteps and ckpt_every must be >= 1");
  const long long V = (long long)cfg->n * cfg->n * cfg->n;
  const int K = std::min(ckpt_every, nsteps);
  *bytes = (size_t)(n_ckpt(nsteps, K) + K) * slot_bytes(V);
  if (K == 1) *bytes += (size_t)nsteps * mid_bytes(V);
  return TUMOR_OK;
}

int tumor_record(tumor_ctx* ctx, int32_t nsteps, int32_t ckpt_every, void* tape, size_t tape_bytes) {
  if (!ctx) return einval("ctx is NULL");
  if (!ctx->adj) {
    g_err = "the context was created without TUMOR_F_ADJOINT";
    return TUMOR_ESTATE;
  }
  if (nsteps < 1 || ckpt_every < 1) return einval("nsteps and ckpt_every must be >= 1");
  if (!tape || (reinterpret_cast<uintptr_t>(tape) & 255u)) return einval("tape must be a 256-byte aligned device pointer");
  size_t need = 0;
  int rc = tumor_tape_bytes(&ctx->cfg, nsteps, ckpt_every, &need);
  if (rc != TUMOR_OK) return rc;
  if (tape_bytes < need) {
    g_err = "tape too small: need " + std::to_string(need) + " bytes";
    return TUMOR_ENOMEM;
  }
  if (ctx->n_ic > 256) return einval("the adjoint supports at most 256 initial-condition centres");
  ctx->tape = static_cast<char*>(tape);
  ctx->tape_bytes = tape_bytes;
  ctx->rec_active = 1;
  ctx->rec_nsteps = nsteps;
  ctx->rec_K = std::min(ckpt_every, nsteps);
  ctx->rec_steps = 0;
  ctx->rev_done = 0;
  ctx->win_start = -1;
  return TUMOR_OK;
}

int tumor_adjoint_step(tumor_ctx* ctx, double* adj, double* grad) {
  if (!ctx) return einval("ctx is NULL");
  if (!adj || !grad) return einval("adj/grad is NULL");
  if (!ctx->rec_active || ctx->rec_steps - ctx->rev_done <= 0) {
    g_err = "no recorded forward step left to reverse";
    return TUMOR_ESTATE;
  }
  return guarded([&]() -> int {
    Ctx& c = *ctx;
    const int m = c.rec_steps - 1 - c.rev_done;
    const int K = c.rec_K;
    if (K == 1 && c.rec_steps == c.rec_nsteps) {
      // Every state and the step's intermediates are on the tape: restore the
      // context as the forward step m left it, then transpose.
      const double* x0 = tape_slot(c, m);
      if (c.flags & TUMOR_F_ADVECTION) {
        // the step's velocity (u^m - u^{m-1}) / dt, from the state it started from
        cplx<double>* u = c.U;
        cplx<double>* up = c.Up;
        c.U = reinterpret_cast<cplx<double>*>(const_cast<double*>(x0) + 8 * c.V);
        c.Up = reinterpret_cast<cplx<double>*>(const_cast<double*>(x0) + 11 * c.V);
        velocity(c);
        c.U = u;
        c.Up = up;
      }
      load_state(c, tape_slot(c, m + 1));  // post-step species and displacements, refreshed coefficients
      load_mid(c, mid_slot(c, m));
      adjoint_core(c, x0, adj, m, grad);
      c.rev_done++;
      return TUMOR_OK;
    }
    const int nck = n_ckpt(c.rec_nsteps, K);
    if (c.win_start < 0 || m < c.win_start || m >= c.win_start + K) {
      // rebuild the window of states X^ws .. X^m from checkpoint m / K
      const int ws = (m / K) * K;
      load_state(c, tape_slot(c, m / K));
      int status = TUMOR_OK;
      for (int j = ws; j <= m; ++j) {
        save_state(c, tape_slot(c, nck + (j - ws)));
        if (j < m) do_step(c, nullptr, status);
      }
      if (status == TUMOR_ENAN) throw Fail(TUMOR_ENAN, "non-finite value while recomputing the forward window");
      c.win_start = ws;
    }
    const double* x0 = tape_slot(c, nck + (m - c.win_start));
    load_state(c, x0);
    int status = TUMOR_OK;
    do_step(c, nullptr, status);
    if (status == TUMOR_ENAN) throw Fail(TUMOR_ENAN, "non-finite value while recomputing the forward step");
    adjoint_core(c, x0, adj, m, grad);
    c.rev_done++;
    return TUMOR_OK;
  });
}

int tumor_kernel_timer(tumor_ctx* ctx, int32_t kernel_class, int32_t enable) {
  if (!ctx) return einval("ctx is NULL");
  if (kernel_class < 0 || kernel_class >= TUMOR_K_COUNT) return einval("unknown kernel class");
  return guarded([&]() -> int {
    Ctx& c = *ctx;
    KTimer*& t = c.timers[kernel_class];
    if (!t) {
      t = new KTimer;
      std::memset(t, 0, sizeof(*t));
      for (int k = 0; k < 2 * kMaxPend; ++k) HIPCHECK(hipEventCreate(&t->ev[k]));
    }
    timer_flush(c, kernel_class, 0x7fffffff);
    t->on = enable ? 1 : 0;
    if (enable) {
      t->launches = 0;
      t->ms = 0.0;
      t->bytes = 0.0;
    }
    return TUMOR_OK;
  });
}

int tumor_kernel_timer_read(tumor_ctx* ctx, int32_t kernel_class, int64_t* launches, double* ms, double* bytes) {
  if (!ctx) return einval("ctx is NULL");
  if (kernel_class < 0 || kernel_class >= TUMOR_K_COUNT) return einval("unknown kernel class");
  return guarded([&]() -> int {
    Ctx& c = *ctx;
    KTimer* t = c.timers[kernel_class];
    if (t) timer_flush(c, kernel_class, 0x7fffffff);
    if (launches) *launches = t ? t->launches : 0;
    if (ms) *ms = t ? t->ms : 0.0;
    if (bytes) *bytes = t ? t->bytes : 0.0;
    return TUMOR_OK;
  });
}

int tumor_substep_timer(tumor_ctx* ctx, int32_t enable) {
  if (!ctx) return einval("ctx is NULL");
  return guarded([&]() -> int {
    Ctx& c = *ctx;
    if (enable && !c.sub_ev[0]) {
      for (int k = 0; k < 6; ++k) HIPCHECK(hipEventCreate(&c.sub_ev[k]));
    }
    c.sub_on = enable != 0;
    for (int k = 0; k < TUMOR_SUB_COUNT; ++k) c.sub_ms[k] = 0.0;
    c.sub_steps = 0;
    return TUMOR_OK;
  });
}

int tumor_substep_timer_read(tumor_ctx* ctx, int64_t* steps, double* ms) {
  if (!ctx) return einval("ctx is NULL");
  if (!steps || !ms) return einval("steps/ms is NULL");
  *steps = ctx->sub_steps;
  for (int k = 0; k < TUMOR_SUB_COUNT; ++k) ms[k] = ctx->sub_ms[k];
  return TUMOR_OK;
}

int tumor_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream) {
  if (!src || !dst) return einval("src/dst is NULL");
  if ((bytes & 15u) != 0) return einval("bytes must be a multiple of 16");
  if ((reinterpret_cast<uintptr_t>(src) & 15u) || (reinterpret_cast<uintptr_t>(dst) & 15u))
    return einval("src and dst must be 16-byte aligned");
  if (bytes >= (size_t(1) << 42)) return einval("bytes out of range");
  return guarded([&]() -> int {
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    tumor::launch_stream_copy(src, dst, (long long)bytes, st);
    HIPCHECK(hipGetLastError());
    return TUMOR_OK;
  });
}

// A snapshot starts with a 256-byte header (magic, grid size, field count) so
// that a snapshot of another grid is refused; the state follows.
constexpr size_t kSnapHeader = 256;
constexpr long long kSnapMagic = 0x54554d4f52534e31LL;  // "TUMORSN1"

int tumor_state_bytes(const tumor_config* cfg, size_t* bytes) {
  if (!bytes) return einval("bytes is NULL");
  if (check_cfg(cfg) != TUMOR_OK) return einval("invalid tumor_config");
  *bytes = kSnapHeader + slot_bytes((long long)cfg->n * cfg->n * cfg->n);
  return TUMOR_OK;
}

int tumor_save_state(tumor_ctx* ctx, void* dst, size_t bytes) {
  if (!ctx) return einval("ctx is NULL");
  if (!dst) return einval("dst is NULL");
  if (bytes < kSnapHeader + slot_bytes(ctx->V)) return einval("snapshot buffer smaller than tumor_state_bytes");
  if (reinterpret_cast<uintptr_t>(dst) & 7u) return einval("dst must be 8-byte aligned");
  return guarded([&]() -> int {
    // the whole header is written (zeros after the four fields), so equal
    // states give byte-identical snapshots
    long long hdr[kSnapHeader / sizeof(long long)] = {kSnapMagic, ctx->n, 14, 0};
    HIPCHECK(hipMemcpyAsync(dst, hdr, sizeof(hdr), hipMemcpyHostToDevice, ctx->st));
    save_state(*ctx, reinterpret_cast<double*>(static_cast<char*>(dst) + kSnapHeader));
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(ctx->st));
    return TUMOR_OK;
  });
}

int tumor_load_state(tumor_ctx* ctx, const void* src, size_t bytes) {
  if (!ctx) return einval("ctx is NULL");
  if (!src) return einval("src is NULL");
  if (bytes < kSnapHeader + slot_bytes(ctx->V)) return einval("snapshot buffer smaller than tumor_state_bytes");
  if (reinterpret_cast<uintptr_t>(src) & 7u) return einval("src must be 8-byte aligned");
  if (ctx->rec_active && (ctx->rec_steps < ctx->rec_nsteps || ctx->rev_done < ctx->rec_steps)) {
    g_err = "a recording or its reverse sweep is in progress; loading a state would invalidate its tape";
    return TUMOR_ESTATE;
  }
  return guarded([&]() -> int {
    long long hdr[4] = {0, 0, 0, 0};
    HIPCHECK(hipMemcpyAsync(hdr, src, sizeof(hdr), hipMemcpyDeviceToHost, ctx->st));
    HIPCHECK(hipStreamSynchronize(ctx->st));
    if (hdr[0] != kSnapMagic || hdr[1] != ctx->n || hdr[2] != 14)
      throw Fail(TUMOR_EINVAL, "not a state snapshot of a grid of this size");
    ctx->rec_active = 0;
    load_state(*ctx, reinterpret_cast<const double*>(static_cast<const char*>(src) + kSnapHeader));
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(ctx->st));
    return TUMOR_OK;
  });
}

void tumor_destroy(tumor_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->st);
  for (int k = 0; k < TUMOR_K_COUNT; ++k) {
    if (!ctx->timers[k]) continue;
    for (int e = 0; e < 2 * kMaxPend; ++e) (void)hipEventDestroy(ctx->timers[k]->ev[e]);
    delete ctx->timers[k];
  }
  for (int k = 0; k < TUMOR_K_COUNT; ++k) ctx->timers[k] = nullptr;
  for (int k = 0; k < 6; ++k)
    if (ctx->sub_ev[k]) (void)hipEventDestroy(ctx->sub_ev[k]);
  if (ctx->static_dev >= 0) {
    // allocation-free context: its storage is the device's static slot
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static[ctx->static_dev].in_use = false;
    return;
  }
  if (ctx->hsv) (void)hipHostFree(ctx->hsv);
  if (ctx->hcs) (void)hipHostFree(ctx->hcs);
  delete[] ctx->ic_host;
  delete ctx;
}

}  // extern "C"
