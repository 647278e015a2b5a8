// Adjoint kernels of the split step (launchers and argument blocks).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace tumor {

// Parameter-gradient accumulators: g[0] rho, g[1] k_w, g[2] k_g, g[3] k_f, g[4] lame_scale.
struct GradScalars {
  double g[8];
  int32_t pad[4];
  // maxima (bits of non-negative doubles, combined by atomic max) that bound the
  // transposed transport's contributions: |lam_k|, |q_k| (k = 0..5), |div v|,
  // |v| (largest component)
  unsigned long long slb[14];
};

struct ReactAdjArgs {
  // forward values of the step
  const double *p_dag, *i_dag, *i_dd, *g_dag, *w_dag, *o_dag;  // reaction inputs (no derivative of the reaction needs n)
  const double *i1, *g1, *w1;                                         // reaction outputs used by O2/edema
  const double *w0, *g0;                                              // step-start tissue (rho_p)
  double rho_w, rho_g;
  // adjoints: L[0..6] = p, i, n, o, l, g, w (in: of the outputs; out: see kernel)
  double* L[7];
  double *idd, *ddb, *rb;
  long long V;
  ReactConsts rc;
};

struct CoefAdjArgs {
  const double *mub, *lamb, *etab;
  const double *p1, *i1, *n1, *g1, *w1, *f1;
  const double* bg;  // static background fraction
  double* L[8];  // p, i, n, o, l, g, w, f
  RefreshConsts fc;
  double inv_scale;
  double* partials;
  GradScalars* gs;
  long long V;
};

struct S0AdjArgs {
  const double *Kb, *rb, *w0, *g0, *f0;
  double *Lw, *Lg, *Lf;
  double k_w, k_g, k_f, rho_w, rho_g;
  double* partials;
  GradScalars* gs;
  long long V;
};

struct SLAdjArgs {
  const double *vx, *vy, *vz, *div;
  const double* q[6];    // p, i, n, g, w, f at step start
  const double* lam[6];  // adjoints of the transported p, i, n, g, w, f
  double* out[6];        // scatter targets (zeroed by the caller)
  double* divb;          // adjoint of div v (zeroed by the caller)
  double* vb[3];         // adjoint of v (zeroed by the caller)
  int n_grid;
  double dt, s;
};

void launch_react_adj(const ReactAdjArgs& a, hipStream_t st);
void launch_coef_adj(const CoefAdjArgs& a, hipStream_t st);
void launch_s0_adj(const S0AdjArgs& a, hipStream_t st);
void launch_force_adj(long long V, double zeta, const double* p, const double* n, const double* gtau,
                      const double* y, double* taub, double* W, hipStream_t st);
void launch_axpy(long long V, double coef, const double* x, double* out, hipStream_t st);
void launch_xpay(long long V, const double* x, double coef, const double* y, double* out, hipStream_t st);
// Transposed transport: bounds pass, scatter into 64-bit fixed-point
// accumulators (out, divb, vb, zeroed by the caller), conversion back to FP64.
// gs->slb must be zero on entry.
void launch_sl_adj(const SLAdjArgs& a, GradScalars* gs, hipStream_t st);
int ic_adj_blocks(int n);
void launch_ic_adj(int n, const double* ic, int n_ic, const double* lam_p, double* part, double* out,
                   hipStream_t st);

}  // namespace tumor
