// Adjoint kernels of the split step (gfx950, FP64).
//
// Each kernel is the transpose of the linearisation of one forward sub-step:
//   k_react_adj : species reaction, oxygen and edema updates (pointwise)
//   k_coef_adj  : Lame / screening mixture -> species adjoints, d/d lame_scale
//   k_s0_adj    : step coefficients K, rho -> w, g, f and d/d(k_w, k_g, k_f, rho)
//   k_force_adj : pointwise part of the force b = zeta tanh(tau) G tau
//   k_sl_adj    : semi-Lagrangian transport (interpolation transpose summed
//                 per brick in LDS, then added to global memory, both in 64-bit
//                 fixed point so that the sums do not depend on the order of the
//                 atomics; velocity sensitivity through X and X*)
//   k_ic_adj    : projections onto the Gaussian initial-condition basis
// Parameter sums use deterministic block partials totalled by a one-block kernel.
#include <algorithm>
#include <climits>
#include <cmath>
#include <stdexcept>

#include "adjoint.hpp"

namespace tumor {

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block partials of v[] (plain stores); k_fin_grad, queued right after the
// kernel, adds their fixed-order totals to gs->g[slot0 + k].
template <int NV>
__device__ void store_grad_partials(double (&v)[NV], double* part) {
  __shared__ double sh[NV][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wave_sum_d(v[k]);
    if (lane == 0) sh[k][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) part[(long long)blockIdx.x * NV + k] = sh[k][0] + sh[k][1] + sh[k][2] + sh[k][3];
  }
}

template <int NV>
__global__ void __launch_bounds__(256) k_fin_grad(GradScalars* gs, const double* part, int nb, int slot0) {
  __shared__ double sh[NV][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double t[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) t[k] = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < NV; ++k) t[k] += part[(long long)b * NV + k];
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wave_sum_d(t[k]);
    if (lane == 0) sh[k][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) gs->g[slot0 + k] += sh[k][0] + sh[k][1] + sh[k][2] + sh[k][3];
  }
}

static inline int rblocks(long long V) {
  long long b = (V + 255) / 256;
  return (int)(b > 1024 ? 1024 : (b < 1 ? 1 : b));
}

// ----------------------------------------------------------- pointwise math
__device__ __forceinline__ double H(double x, double eps) { return 1.0 / (1.0 + exp(-2.0 * x / eps)); }
__device__ __forceinline__ double dH(double x, double eps) {
  const double h = H(x, eps);
  return (2.0 / eps) * h * (1.0 - h);
}
__device__ __forceinline__ void logistic_partials(double y, double r, double t, double& ly, double& lr,
                                                  double& val) {
  const double e = exp(r * t);
  const double D = 1.0 + y * (e - 1.0);
  ly = e / (D * D);
  lr = t * e * y * (1.0 - y) / (D * D);
  val = y * e / D;
}

// Reaction + oxygen + edema transpose.  L[] are the adjoints of the step's
// outputs p', i', n', o', l', g', w' on entry; on exit L[P], L[N], L[G], L[W]
// hold the adjoints of p, n, g, w after transport, L[O] that of o after
// diffusion, L[L] that of l after diffusion; idd = adjoint of i after
// diffusion (including the dD term), ddb = adjoint of dD, rb = adjoint of
// rho_p + rho_inv_frac * adjoint of rho_i.
__global__ void __launch_bounds__(256) k_react_adj(ReactAdjArgs a) {
  const ReactConsts& rc = a.rc;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < a.V;
       v += (long long)gridDim.x * blockDim.x) {
    const double dt = rc.dt, eps = rc.eps;
    const double p = a.p_dag[v], idag = a.i_dag[v], i = a.i_dd[v], n = a.n_dag[v], g = a.g_dag[v],
                 w = a.w_dag[v], o = a.o_dag[v];
    const double i1 = a.i1[v], g1 = a.g1[v], w1 = a.w1[v];
    const double rho_p = a.rho_w * a.w0[v] + a.rho_g * a.g0[v];
    const double rho_i = rc.rho_inv_frac * rho_p;
    double Pb = a.L[0][v], Ib = a.L[1][v], Nb = a.L[2][v], Ob = a.L[3][v], Lb = a.L[4][v], Gb = a.L[5][v],
           Wb = a.L[6][v];
    // edema: l' = l + dt (delta_e i'/(i'+dh)(1-i') - delta_l l)
    double ldag_b = Lb;
    if (rc.edema) {
      ldag_b = Lb * (1.0 - dt * rc.delta_l);
      const double dh = rc.delta_half;
      Ib += Lb * dt * rc.delta_e * (dh * (1.0 - i1) / ((i1 + dh) * (i1 + dh)) - i1 / (i1 + dh));
    }
    // oxygen: o' = o + dt (-delta_p p' + delta_s (o_heal - o)(g' + w'))
    double odag_b = Ob * (1.0 - dt * rc.delta_s * (g1 + w1));
    Pb += Ob * (-dt * rc.delta_p);
    const double gwo = Ob * dt * rc.delta_s * (rc.o_heal - o);
    Gb += gwo;
    Wb += gwo;
    // species reaction
    const double Ha = H(rc.o_inv - o, eps);
    const double alpha = rc.alpha0 * Ha;
    const double alpha_o = -rc.alpha0 * dH(rc.o_inv - o, eps);
    const double Hb = H(rc.sigma_b - p - i, eps);
    const double beta = rc.beta0 * Hb * o;
    const double beta_pi = -rc.beta0 * dH(rc.sigma_b - p - i, eps) * o;
    const double beta_o = rc.beta0 * Hb;
    const double h = rc.gamma * H(rc.o_hyp - o, eps);
    const double h_o = -rc.gamma * dH(rc.o_hyp - o, eps);
    double kap = (o - rc.o_mit) / (rc.o_inv - rc.o_mit);
    kap = kap < 0.0 ? 0.0 : (kap > 1.0 ? 1.0 : kap);
    const double kap_o = (o >= rc.o_mit && o <= rc.o_inv) ? 1.0 / (rc.o_inv - rc.o_mit) : 0.0;
    double Lpy, Lpr, Lp, Liy, Lir, Li;
    logistic_partials(p, rho_p * kap, dt, Lpy, Lpr, Lp);
    logistic_partials(i, rho_i * kap, dt, Liy, Lir, Li);
    const double dD = i - idag;
    const double S = dD + (Lp - p) + (Li - i);
    const double gw = g + w;
    const bool small = gw < 1e-12;
    const double phig = small ? 0.5 : g / gw;
    const double phiw = small ? 0.5 : w / gw;
    const double inv2 = small ? 0.0 : 1.0 / (gw * gw);
    const double dphig_g = w * inv2, dphig_w = -g * inv2, dphiw_g = -w * inv2, dphiw_w = g * inv2;
    const double Sb = -phig * Gb - phiw * Wb;
    const double tot = p + i + g + w;
    const double p_b = Pb * (Lpy + dt * (-alpha + beta_pi * i - h)) + Ib * dt * (alpha - beta_pi * i) +
                       Nb * dt * h + Sb * (Lpy - 1.0);
    const double i_b = Pb * dt * (beta + beta_pi * i) + Ib * (Liy + dt * (-beta - beta_pi * i - h)) + Nb * dt * h +
                       Sb * (Liy - 1.0);
    const double g_b = Nb * dt * h + Gb * (1.0 - dphig_g * S - dt * h) + Wb * (-dphiw_g * S);
    const double w_b = Nb * dt * h + Gb * (-dphig_w * S) + Wb * (1.0 - dphiw_w * S - dt * h);
    const double o_b = Pb * (Lpr * rho_p * kap_o + dt * (-alpha_o * p + beta_o * i - h_o * p)) +
                       Ib * (Lir * rho_i * kap_o + dt * (alpha_o * p - beta_o * i - h_o * i)) +
                       Nb * dt * h_o * tot + Sb * (Lpr * rho_p + Lir * rho_i) * kap_o - Gb * dt * h_o * g -
                       Wb * dt * h_o * w;
    const double rp_b = (Pb + Sb) * Lpr * kap;
    const double ri_b = (Ib + Sb) * Lir * kap;
    a.L[0][v] = p_b;
    a.L[2][v] = Nb;
    a.L[5][v] = g_b;
    a.L[6][v] = w_b;
    a.L[3][v] = odag_b + o_b;
    a.L[4][v] = ldag_b;
    a.idd[v] = i_b + Sb;
    a.ddb[v] = Sb;
    a.rb[v] = rp_b + rc.rho_inv_frac * ri_b;
  }
}

// Lame / screening mixture transposed (S5) and d/d lame_scale.
__global__ void __launch_bounds__(256) k_coef_adj(CoefAdjArgs a) {
  double acc[1] = {0.0};
  const RefreshConsts& fc = a.fc;  // scaled by lame_scale
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < a.V;
       v += (long long)gridDim.x * blockDim.x) {
    const double mb = a.mub[v], lb = a.lamb[v], eb = a.etab[v];
    const double p = a.p1[v], i = a.i1[v], n = a.n1[v], g = a.g1[v], w = a.w1[v], f = a.f1[v];
    const double tau = p + i + n;
    const double tb = fc.mu_t * mb + fc.la_t * lb + fc.eta_t * eb;
    a.L[0][v] += tb;
    a.L[1][v] += tb;
    a.L[2][v] += tb;
    a.L[5][v] += fc.mu_g * mb + fc.la_g * lb + fc.eta_h * eb;
    a.L[6][v] += fc.mu_w * mb + fc.la_w * lb + fc.eta_h * eb;
    a.L[7][v] += fc.mu_f * mb + fc.la_f * lb + fc.eta_h * eb;
    const double b = a.bg[v];
    const double mu = fc.mu_w * w + fc.mu_g * g + fc.mu_f * f + fc.mu_t * tau + fc.mu_b * b;
    const double la = fc.la_w * w + fc.la_g * g + fc.la_f * f + fc.la_t * tau + fc.la_b * b;
    acc[0] += (mu * mb + la * lb) * a.inv_scale;
  }
  store_grad_partials<1>(acc, a.partials);
}

// Step coefficients (S0) transposed: K = k_w w + k_g g + k_f f, rho_p = rho_w w + rho_g g.
__global__ void __launch_bounds__(256) k_s0_adj(S0AdjArgs a) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < a.V;
       v += (long long)gridDim.x * blockDim.x) {
    const double kb = a.Kb[v], rb = a.rb[v];
    const double w0 = a.w0[v], g0 = a.g0[v], f0 = a.f0[v];
    a.Lw[v] += a.k_w * kb + a.rho_w * rb;
    a.Lg[v] += a.k_g * kb + a.rho_g * rb;
    a.Lf[v] += a.k_f * kb;
    acc[0] += (w0 + g0) * rb;
    acc[1] += w0 * kb;
    acc[2] += g0 * kb;
    acc[3] += f0 * kb;
  }
  store_grad_partials<4>(acc, a.partials);
}

// Force b = zeta tanh(tau) G tau, tau = p + n, with b_bar_a = -y_a:
// taub -= zeta sech^2(tau) (G_a tau) y_a ;  W_a = -zeta tanh(tau) y_a.
__global__ void k_force_adj(long long V, double zeta, const double* p, const double* n, const double* gtau,
                            const double* y, double* taub, double* W) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const double t = tanh(p[v] + n[v]);
  taub[v] -= zeta * (1.0 - t * t) * gtau[v] * y[v];
  W[v] = -zeta * t * y[v];
}

__global__ void k_acc_prod(long long V, double coef, const double* x, const double* y, double* out) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < V) out[v] += coef * x[v] * y[v];
}

__global__ void k_axpy(long long V, double coef, const double* x, double* out) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < V) out[v] += coef * x[v];
}

// out = x + coef * y
__global__ void k_xpay(long long V, const double* x, double coef, const double* y, double* out) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < V) out[v] = x[v] + coef * y[v];
}

// ------------------------------------------------------- semi-Lagrangian
__device__ __forceinline__ void lw4(double t, double (&w)[4], double (&d)[4]) {
  w[0] = -t * (t - 1.0) * (t - 2.0) / 6.0;
  w[1] = (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0;
  w[2] = -(t + 1.0) * t * (t - 2.0) / 2.0;
  w[3] = (t + 1.0) * t * (t - 1.0) / 6.0;
  d[0] = -(3.0 * t * t - 6.0 * t + 2.0) / 6.0;
  d[1] = (3.0 * t * t - 4.0 * t - 1.0) / 2.0;
  d[2] = -(3.0 * t * t - 2.0 * t - 2.0) / 2.0;
  d[3] = (3.0 * t * t - 1.0) / 6.0;
}

struct Stencil {
  int ix, iy, iz;
  double wx[4], wy[4], wz[4], dx[4], dy[4], dz[4];
  __device__ __forceinline__ void set(double jx, double jy, double jz) {
    const double bx = floor(jx), by = floor(jy), bz = floor(jz);
    lw4(jx - bx, wx, dx);
    lw4(jy - by, wy, dy);
    lw4(jz - bz, wz, dz);
    ix = (int)(long long)bx;
    iy = (int)(long long)by;
    iz = (int)(long long)bz;
  }
};

// Value and gradient (d/dj along x, y, z) of NF interpolants at one stencil.
template <int NF>
__device__ __forceinline__ void gather_grad(const Stencil& s, const double* const (&q)[NF], int n,
                                            double (&val)[NF], double (&gx)[NF], double (&gy)[NF],
                                            double (&gz)[NF]) {
  const int m = n - 1;
#pragma unroll
  for (int f = 0; f < NF; ++f) val[f] = gx[f] = gy[f] = gz[f] = 0.0;
  // the 16 (z, y) rows stay rolled: unrolled, they hold far more loads in
  // flight than the register file has room for
#pragma unroll 1
  for (int c = 0; c < 4; ++c) {
    const long long zo = (long long)((s.iz + c - 1) & m) * n * n;
#pragma unroll 1
    for (int b = 0; b < 4; ++b) {
      const long long yo = zo + (long long)((s.iy + b - 1) & m) * n;
      const double wzy = s.wz[c] * s.wy[b], dzy = s.dz[c] * s.wy[b], wzdy = s.wz[c] * s.dy[b];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const long long idx = yo + ((s.ix + a - 1) & m);
        const double w = wzy * s.wx[a], wgx = wzy * s.dx[a], wgy = wzdy * s.wx[a], wgz = dzy * s.wx[a];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          const double qv = q[f][idx];
          val[f] += w * qv;
          gx[f] += wgx * qv;
          gy[f] += wgy * qv;
          gz[f] += wgz * qv;
        }
      }
    }
  }
}

// ---- fixed-point accumulation of the transposed interpolation
// Every contribution w * val to a node is rounded to a 64-bit integer at a
// per-field power-of-two scale and summed with integer atomics, which are
// exact and commutative: the result does not depend on the order in which
// threads and blocks add, so the transpose is bitwise reproducible.  The
// scale puts an a-priori bound B of |w * val| (|w| <= 1 for the cubic Lagrange
// weights on [0, 1)) at 2^47, so a node can take 2^16 contributions of the
// bound without overflow; the rounding error of one contribution is at most
// 2^-48 B.
constexpr int kFixBits = 47;

__device__ __forceinline__ long long to_fix(double v, double scale) { return __double2ll_rn(v * scale); }

__device__ __forceinline__ void fix_add(double* acc, long long q) {
  atomicAdd(reinterpret_cast<unsigned long long*>(acc), static_cast<unsigned long long>(q));
}

template <int NF>
__device__ __forceinline__ void scatter(const Stencil& s, double* const (&out)[NF], const double (&val)[NF], int n,
                                        const double (&scale)[NF]) {
  const int m = n - 1;
#pragma unroll 1
  for (int c = 0; c < 4; ++c) {
    const long long zo = (long long)((s.iz + c - 1) & m) * n * n;
#pragma unroll 1
    for (int b = 0; b < 4; ++b) {
      const long long yo = zo + (long long)((s.iy + b - 1) & m) * n;
      const double wzy = s.wz[c] * s.wy[b];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const long long idx = yo + ((s.ix + a - 1) & m);
        const double w = wzy * s.wx[a];
#pragma unroll
        for (int f = 0; f < NF; ++f) fix_add(out[f] + idx, to_fix(w * val[f], scale[f]));
      }
    }
  }
}

// One 16 x 4 x 4 brick of arrival voxels per 256-thread block (n >= 16, so the
// bricks tile the grid), bricks laid out x fastest, and consecutive block
// indices spread over the 8 XCDs so that each XCD sweeps a contiguous slab.
constexpr int kSlAdjBX = 16, kSlAdjBY = 4, kSlAdjBZ = 4;
// LDS accumulation tile for the transposed interpolation (64-bit fixed point).  A brick's
// stencils span (16 + 3 + dx) x (4 + 3 + dy) x (4 + 3 + dz) nodes, dx, dy, dz
// the spread of its departure cells; 2048 covers a spread of 2 cells per axis.
constexpr int kSlAdjTile = 2048;

// Transposed interpolation of NF values per voxel of a block: each tap's
// contribution w * val[f] goes to the node it was read from.  Contributions
// are first summed in an LDS tile over the bounding box of the block's
// stencils (LDS atomics), then each tile node is added to global memory with
// one atomic, one field at a time.  A block whose box exceeds the tile adds
// every contribution with a global atomic instead.  All sums are 64-bit fixed
// point (scale[f] per field), so both paths give the same integers.  Called by
// all threads of the block (block-uniform control flow).
template <int NF>
__device__ void scatter_tiled(const Stencil& s, double* const (&out)[NF], const double (&val)[NF], int n,
                              const double (&scale)[NF], long long* tile, int* box) {
  __syncthreads();  // every thread is done with box from a previous call
  if (threadIdx.x == 0) {
    box[0] = box[1] = box[2] = INT_MAX;
    box[3] = box[4] = box[5] = INT_MIN;
  }
  __syncthreads();
  atomicMin(&box[0], s.ix);
  atomicMin(&box[1], s.iy);
  atomicMin(&box[2], s.iz);
  atomicMax(&box[3], s.ix);
  atomicMax(&box[4], s.iy);
  atomicMax(&box[5], s.iz);
  __syncthreads();
  const int x0 = box[0], y0 = box[1], z0 = box[2];
  const long long DX = (long long)box[3] - x0 + 4, DY = (long long)box[4] - y0 + 4, DZ = (long long)box[5] - z0 + 4;
  if (DX * DY * DZ > kSlAdjTile) {
    scatter<NF>(s, out, val, n, scale);
    return;
  }
  const int m = n - 1;
  const int dxn = (int)DX, dyn = (int)DY, cnt = (int)(DX * DY * DZ);
  // tile coordinates of the stencil's first node (x0 - 1, y0 - 1, z0 - 1 is the tile origin)
  const int bx = s.ix - x0, by = s.iy - y0, bz = s.iz - z0;
  for (int f = 0; f < NF; ++f) {
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) tile[k] = 0;
    __syncthreads();
#pragma unroll 1
    for (int c = 0; c < 4; ++c) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const double wzy = s.wz[c] * s.wy[b];
        const int row = ((bz + c) * dyn + (by + b)) * dxn + bx;
#pragma unroll
        for (int a = 0; a < 4; ++a)
          atomicAdd(reinterpret_cast<unsigned long long*>(&tile[row + a]),
                    static_cast<unsigned long long>(to_fix(wzy * s.wx[a] * val[f], scale[f])));
      }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
      const long long t = tile[k];
      if (t != 0) {
        const int tx = k % dxn, ty = (k / dxn) % dyn, tz = k / (dxn * dyn);
        const long long idx =
            ((long long)((z0 - 1 + tz) & m) * n + ((y0 - 1 + ty) & m)) * n + ((x0 - 1 + tx) & m);
        fix_add(out[f] + idx, t);
      }
    }
    __syncthreads();
  }
}

// Maxima that bound the transpose's contributions (one atomic max per block
// and quantity on the bits of the non-negative doubles; NaN reads as +inf).
__global__ void __launch_bounds__(256) k_sl_adj_bounds(SLAdjArgs a, GradScalars* gs) {
  const long long V = (long long)a.n_grid * a.n_grid * a.n_grid;
  double m[14];
#pragma unroll
  for (int k = 0; k < 14; ++k) m[k] = 0.0;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      m[k] = fmax(m[k], fabs(a.lam[k][v]));
      m[6 + k] = fmax(m[6 + k], fabs(a.q[k][v]));
    }
    m[12] = fmax(m[12], fabs(a.div[v]));
    m[13] = fmax(m[13], fmax(fabs(a.vx[v]), fmax(fabs(a.vy[v]), fabs(a.vz[v]))));
  }
  __shared__ double sh[14][4];
#pragma unroll
  for (int k = 0; k < 14; ++k) {
    double t = m[k];
    if (!(t >= 0.0)) t = INFINITY;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t = fmax(t, __shfl_xor(t, off, 64));
    if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = t;
  }
  __syncthreads();
  if (threadIdx.x < 14) {
    const int k = threadIdx.x;
    const double t = fmax(fmax(sh[k][0], sh[k][1]), fmax(sh[k][2], sh[k][3]));
    atomicMax(&gs->slb[k], (unsigned long long)__double_as_longlong(t));
  }
}

// Fixed-point scales of the ten accumulated fields (out[0..5], divb, vb[0..2])
// from a-priori bounds of their contributions (grid-index units).  With A_k,
// Q_k the maxima of |lam_k| and |q_k|, D of |div v|, Vm of |v|, and the
// Lebesgue constants of tricubic Lagrange interpolation, Lam = 1.25^3 for
// values and Ld = 2.334 * 1.25^2 for one first derivative (the maxima over a
// cell of sum |l_i| and sum |l_i'| in 1-D are 1.25 and 7/3):
//   |cfac| <= Cf = 1 + dt/2 (Lam + 1) D + dt^2/2 Lam D^2,
//   |bar_k| <= A_k Cf (k < 5), |bar_5| <= A_5,
//   |cbar| <= Cb = Lam sum_{k<5} A_k Q_k, |bar_6| <= Cb (dt/2 + dt^2/2 D),
//   |ddirect| <= Cb (dt/2 + dt^2/2 Lam D),
//   |Jb| <= J = Ld (sum_{k<6} |bar_k| Q_k + |bar_6| D), |vsb| <= s J / 2,
//   |vown| <= s J / 2 + 3 s (s J / 2) Ld Vm.
// scale = 2^(kFixBits - e) with 2^e >= bound.  A non-finite bound leaves
// finite = false (the finishing pass then writes NaN).
__device__ __forceinline__ void sl_adj_scales(const GradScalars* gs, double dt, double s, double (&scale)[10],
                                              bool& finite) {
  double mx[14];
#pragma unroll
  for (int k = 0; k < 14; ++k) mx[k] = __longlong_as_double((long long)gs->slb[k]);
  const double Lam = 1.953125, Ld = 3.6459, D = mx[12], Vm = mx[13];
  const double Cf = 1.0 + 0.5 * dt * (Lam + 1.0) * D + 0.5 * dt * dt * Lam * D * D;
  double bnd[10], barm[7];
  double Cb = 0.0;
  for (int k = 0; k < 5; ++k) {
    barm[k] = mx[k] * Cf;
    Cb += mx[k] * mx[6 + k];
  }
  Cb *= Lam;
  barm[5] = mx[5];
  barm[6] = Cb * (0.5 * dt + 0.5 * dt * dt * D);
  const double dd = Cb * (0.5 * dt + 0.5 * dt * dt * Lam * D);
  double J = barm[6] * D;
  for (int k = 0; k < 6; ++k) J += barm[k] * mx[6 + k];
  J *= Ld;
  const double vsb = 0.5 * s * J;
  for (int k = 0; k < 6; ++k) bnd[k] = barm[k];
  bnd[6] = fmax(barm[6], dd);
  const double vown = vsb + 3.0 * s * vsb * Ld * Vm;
  for (int k = 7; k < 10; ++k) bnd[k] = fmax(vsb, vown);
  finite = true;
  for (int k = 0; k < 10; ++k) {
    const double b = bnd[k];
    if (!(b < INFINITY)) {
      finite = false;
      scale[k] = 1.0;
    } else if (b > 0.0) {
      const int e = max(ilogb(b) + 1, -900);  // 2^e > b
      scale[k] = ldexp(1.0, kFixBits - e);
    } else {
      scale[k] = 1.0;  // every contribution is zero
    }
  }
}

// Fixed point back to FP64 in place (ten fields of V values).
__global__ void __launch_bounds__(256) k_sl_adj_finish(SLAdjArgs a, const GradScalars* gs) {
  double scale[10];
  bool finite;
  sl_adj_scales(gs, a.dt, a.s, scale, finite);
  double* const f[10] = {a.out[0], a.out[1], a.out[2], a.out[3], a.out[4], a.out[5], a.divb,
                         a.vb[0], a.vb[1], a.vb[2]};
  const long long V = (long long)a.n_grid * a.n_grid * a.n_grid;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      const long long q = __double_as_longlong(f[k][v]);
      f[k][v] = finite ? (double)q / scale[k] : NAN;
    }
  }
}

__global__ void __launch_bounds__(256) k_sl_adj(SLAdjArgs a, const GradScalars* gs) {
  __shared__ long long tile[kSlAdjTile];
  __shared__ int box[6];
  double scale[10];
  bool finite;
  sl_adj_scales(gs, a.dt, a.s, scale, finite);
  const int n = a.n_grid;
  const int nbx = n / kSlAdjBX, nby = n / kSlAdjBY;
  const int nb = (int)gridDim.x;
  const int blk = (int)(blockIdx.x % 8) * (nb / 8) + (int)(blockIdx.x / 8);
  const int jx = (blk % nbx) * kSlAdjBX + (int)(threadIdx.x % kSlAdjBX);
  const int jy = ((blk / nbx) % nby) * kSlAdjBY + (int)((threadIdx.x / kSlAdjBX) % kSlAdjBY);
  const int jz = (blk / (nbx * nby)) * kSlAdjBZ + (int)(threadIdx.x / (kSlAdjBX * kSlAdjBY));
  const long long v = ((long long)jz * n + jy) * n + jx;
  const double s = a.s, dt = a.dt;
  const double vx = a.vx[v], vy = a.vy[v], vz = a.vz[v], d0 = a.div[v];
  // X* and v(X*)
  Stencil st_s;
  st_s.set(jx - s * vx, jy - s * vy, jz - s * vz);
  const double* const vel[3] = {a.vx, a.vy, a.vz};
  double vs[3], vsx[3], vsy[3], vsz[3];
  gather_grad<3>(st_s, vel, n, vs, vsx, vsy, vsz);
  // X and the fields there
  Stencil st;
  st.set(jx - 0.5 * s * (vx + vs[0]), jy - 0.5 * s * (vy + vs[1]), jz - 0.5 * s * (vz + vs[2]));
  const double* const fl[7] = {a.q[0], a.q[1], a.q[2], a.q[3], a.q[4], a.q[5], a.div};
  double q[7], qx[7], qy[7], qz[7];
  gather_grad<7>(st, fl, n, q, qx, qy, qz);
  const double dX = q[6];
  const double cfac = 1.0 - 0.5 * dt * (dX + d0) + 0.5 * dt * dt * dX * d0;
  double bar[7];
  double cbar = 0.0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double lam = a.lam[k][v];
    cbar += lam * q[k];
    bar[k] = lam * cfac;
  }
  bar[5] = a.lam[5][v];
  bar[6] = cbar * (-0.5 * dt + 0.5 * dt * dt * d0);
  const double ddirect = cbar * (-0.5 * dt + 0.5 * dt * dt * dX);
  double Jb[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    Jb[0] += bar[k] * qx[k];
    Jb[1] += bar[k] * qy[k];
    Jb[2] += bar[k] * qz[k];
  }
  double* const outs[7] = {a.out[0], a.out[1], a.out[2], a.out[3], a.out[4], a.out[5], a.divb};
  const double sc7[7] = {scale[0], scale[1], scale[2], scale[3], scale[4], scale[5], scale[6]};
  scatter_tiled<7>(st, outs, bar, n, sc7, tile, box);
  fix_add(a.divb + v, to_fix(ddirect, scale[6]));
  // X = x - s/2 (v + v*), v* = I[v](X*), X* = x - s v
  double vsb[3], vown[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    vsb[b] = -0.5 * s * Jb[b];
    vown[b] = -0.5 * s * Jb[b];
  }
  double Jsb[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    Jsb[0] += vsb[b] * vsx[b];
    Jsb[1] += vsb[b] * vsy[b];
    Jsb[2] += vsb[b] * vsz[b];
  }
#pragma unroll
  for (int b = 0; b < 3; ++b) vown[b] += -s * Jsb[b];
  double* const vb[3] = {a.vb[0], a.vb[1], a.vb[2]};
  const double sc3[3] = {scale[7], scale[8], scale[9]};
  scatter_tiled<3>(st_s, vb, vsb, n, sc3, tile, box);
#pragma unroll
  for (int b = 0; b < 3; ++b) fix_add(a.vb[b] + v, to_fix(vown[b], scale[7 + b]));
}

// ------------------------------------------------------ initial condition
// part[k * nb + block] = sum over the block's voxels of phi_k * lam_p.
__global__ void __launch_bounds__(256) k_ic_adj(int n, const double* ic, int n_ic, const double* lam_p,
                                                double* part) {
  const long long V = (long long)n * n * n;
  const int k = blockIdx.y;
  const double h = 2.0 * M_PI / n, twopi = 2.0 * M_PI;
  const double* c = ic + 5 * k;
  double acc = 0.0;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < V;
       v += (long long)gridDim.x * blockDim.x) {
    const int jx = (int)(v % n), jy = (int)((v / n) % n), jz = (int)(v / ((long long)n * n));
    double dx = h * jx - c[0], dy = h * jy - c[1], dz = h * jz - c[2];
    dx -= twopi * rint(dx / twopi);
    dy -= twopi * rint(dy / twopi);
    dz -= twopi * rint(dz / twopi);
    const double d2 = dz * dz + dy * dy + dx * dx;
    acc += exp(-d2 / (2.0 * c[3] * c[3])) * lam_p[v];
  }
  __shared__ double sh[4];
  const double s = wave_sum_d(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[(long long)k * gridDim.x + blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void k_ic_adj_sum(const double* part, int nb, int n_ic, double* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_ic) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(long long)k * nb + b];
  out[k] = s;
}

// ------------------------------------------------------------- launchers
static inline unsigned pw_blocks(long long V) { return (unsigned)((V + 255) / 256); }

void launch_react_adj(const ReactAdjArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_react_adj, dim3(rblocks(a.V)), dim3(256), 0, st, a);
}
void launch_coef_adj(const CoefAdjArgs& a, hipStream_t st) {
  const int nb = rblocks(a.V);
  hipLaunchKernelGGL(k_coef_adj, dim3(nb), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_fin_grad<1>, dim3(1), dim3(256), 0, st, a.gs, a.partials, nb, 4);
}
void launch_s0_adj(const S0AdjArgs& a, hipStream_t st) {
  const int nb = rblocks(a.V);
  hipLaunchKernelGGL(k_s0_adj, dim3(nb), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_fin_grad<4>, dim3(1), dim3(256), 0, st, a.gs, a.partials, nb, 0);
}
void launch_force_adj(long long V, double zeta, const double* p, const double* n, const double* gtau,
                      const double* y, double* taub, double* W, hipStream_t st) {
  hipLaunchKernelGGL(k_force_adj, dim3(pw_blocks(V)), dim3(256), 0, st, V, zeta, p, n, gtau, y, taub, W);
}
void launch_acc_prod(long long V, double coef, const double* x, const double* y, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_acc_prod, dim3(pw_blocks(V)), dim3(256), 0, st, V, coef, x, y, out);
}
void launch_axpy(long long V, double coef, const double* x, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3(pw_blocks(V)), dim3(256), 0, st, V, coef, x, out);
}
void launch_xpay(long long V, const double* x, double coef, const double* y, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_xpay, dim3(pw_blocks(V)), dim3(256), 0, st, V, x, coef, y, out);
}
void launch_sl_adj(const SLAdjArgs& a, GradScalars* gs, hipStream_t st) {
  const int n = a.n_grid;
  if (n < 16 || (n & (n - 1)) != 0) throw std::runtime_error("k_sl_adj: grid size must be a power of two >= 16");
  const long long V = (long long)n * n * n;
  const unsigned pw = (unsigned)std::min<long long>(V / 256, 2048);
  hipLaunchKernelGGL(k_sl_adj_bounds, dim3(pw), dim3(256), 0, st, a, gs);
  // one 16 x 4 x 4 brick per block; n^3 / 256 is a multiple of 8 for n >= 16
  const long long nb = V / (kSlAdjBX * kSlAdjBY * kSlAdjBZ);
  hipLaunchKernelGGL(k_sl_adj, dim3((unsigned)nb), dim3(kSlAdjBX * kSlAdjBY * kSlAdjBZ), 0, st, a,
                     static_cast<const GradScalars*>(gs));
  hipLaunchKernelGGL(k_sl_adj_finish, dim3(pw), dim3(256), 0, st, a, static_cast<const GradScalars*>(gs));
}
int ic_adj_blocks(int n) { return rblocks((long long)n * n * n); }
void launch_ic_adj(int n, const double* ic, int n_ic, const double* lam_p, double* part, double* out,
                   hipStream_t st) {
  if (n_ic <= 0) return;
  const int nb = ic_adj_blocks(n);
  hipLaunchKernelGGL(k_ic_adj, dim3(nb, n_ic), dim3(256), 0, st, n, ic, n_ic, lam_p, part);
  hipLaunchKernelGGL(k_ic_adj_sum, dim3((n_ic + 63) / 64), dim3(64), 0, st, part, nb, n_ic, out);
}

}  // namespace tumor
