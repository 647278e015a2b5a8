// Adjoint kernels of the split step (gfx950, FP64).
//
// Each kernel is the transpose of the linearisation of one forward sub-step:
//   k_react_adj : species reaction, oxygen and edema updates (pointwise)
//   k_coef_adj  : Lame / screening mixture -> species adjoints, d/d lame_scale
//   k_s0_adj    : step coefficients K, rho -> w, g, f and d/d(k_w, k_g, k_f, rho)
//   k_force_adj : pointwise part of the force b = zeta tanh(tau) G tau
//   k_sl_adj    : semi-Lagrangian transport (gathers at X* and X from LDS
//                 halo tiles; interpolation transpose summed per brick in LDS,
//                 then added to global memory, both in 64-bit fixed point so
//                 that the sums do not depend on the order of the atomics;
//                 velocity sensitivity through X and X*)
//   k_ic_adj    : projections onto the Gaussian initial-condition basis
// Parameter sums use deterministic block partials totalled by a one-block kernel.
#include <algorithm>
#include <climits>
#include <cmath>
#include <stdexcept>

#include "adjoint.hpp"
#include "sl_tile.hpp"

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
    const double p = a.p_dag[v], idag = a.i_dag[v], i = a.i_dd[v], g = a.g_dag[v],
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
// Cubic Lagrange weights of the nodes j-1 .. j+2 at offset t in [0, 1), and
// their derivatives in t.
__device__ __forceinline__ void lw4(double t, double (&w)[4]) {
  w[0] = -t * (t - 1.0) * (t - 2.0) / 6.0;
  w[1] = (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0;
  w[2] = -(t + 1.0) * t * (t - 2.0) / 2.0;
  w[3] = (t + 1.0) * t * (t - 1.0) / 6.0;
}
__device__ __forceinline__ void dlw4(double t, double (&d)[4]) {
  d[0] = -(3.0 * t * t - 6.0 * t + 2.0) / 6.0;
  d[1] = (3.0 * t * t - 4.0 * t - 1.0) / 2.0;
  d[2] = -(3.0 * t * t - 2.0 * t - 2.0) / 2.0;
  d[3] = (3.0 * t * t - 1.0) / 6.0;
}

// Tricubic stencil of a point in grid-index units: base node and weights.
struct Stencil {
  int ix, iy, iz;
  double wx[4], wy[4], wz[4];
  __device__ __forceinline__ void set(double jx, double jy, double jz) {
    const double bx = floor(jx), by = floor(jy), bz = floor(jz);
    lw4(jx - bx, wx);
    lw4(jy - by, wy);
    lw4(jz - bz, wz);
    ix = (int)(long long)bx;
    iy = (int)(long long)by;
    iz = (int)(long long)bz;
  }
};

// The same with the derivative weights, for value-and-gradient gathers.
struct StencilD : Stencil {
  double dx[4], dy[4], dz[4];
  __device__ __forceinline__ void set(double jx, double jy, double jz) {
    Stencil::set(jx, jy, jz);
    dlw4(jx - floor(jx), dx);
    dlw4(jy - floor(jy), dy);
    dlw4(jz - floor(jz), dz);
  }
};

// w[i] for a runtime i in 0..3 by selects, so that rolled loops do not put
// the weight arrays in scratch memory.
__device__ __forceinline__ double pick4(const double (&w)[4], int i) {
  return i == 0 ? w[0] : (i == 1 ? w[1] : (i == 2 ? w[2] : w[3]));
}

// Visit the 64 nodes of a stencil: fn(idx, w, wgx, wgy, wgz) with the value
// weight and the three derivative weights (d/dj along x, y, z) of the node.
// The 16 (z, y) rows stay rolled: unrolled, they hold far more loads in
// flight than the register file has room for.
template <typename Fn>
__device__ __forceinline__ void for_taps(const StencilD& s, int n, Fn fn) {
  const int m = n - 1;
#pragma unroll 1
  for (int r = 0; r < 16; ++r) {
    const int c = r >> 2, b = r & 3;
    const long long yo = ((long long)((s.iz + c - 1) & m) * n + ((s.iy + b - 1) & m)) * n;
    const double wz = pick4(s.wz, c), dz = pick4(s.dz, c), wy = pick4(s.wy, b), dy = pick4(s.dy, b);
    const double wzy = wz * wy, dzy = dz * wy, wzdy = wz * dy;
#pragma unroll
    for (int a = 0; a < 4; ++a)
      fn(yo + ((s.ix + a - 1) & m), wzy * s.wx[a], wzy * s.dx[a], wzdy * s.wx[a], dzy * s.wx[a]);
  }
}

// Value and gradient of the three velocity interpolants at one stencil:
// val[b] = I[v_b], g[b][a] = d/dj_a I[v_b].
__device__ __forceinline__ void gather_vel(const StencilD& s, const double* __restrict__ vx,
                                           const double* __restrict__ vy, const double* __restrict__ vz, int n,
                                           double (&val)[3], double (&g)[3][3]) {
#pragma unroll
  for (int b = 0; b < 3; ++b) val[b] = g[b][0] = g[b][1] = g[b][2] = 0.0;
  for_taps(s, n, [&](long long idx, double w, double wgx, double wgy, double wgz) {
    const double q[3] = {vx[idx], vy[idx], vz[idx]};
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      val[b] += w * q[b];
      g[b][0] += wgx * q[b];
      g[b][1] += wgy * q[b];
      g[b][2] += wgz * q[b];
    }
  });
}

// The interpolants that the transpose needs at the departure point X, with
// the arrival voxel's adjoints lam (constant over the stencil) folded in
// before the sums: e = I[sum_{k<5} lam_k q_k] and its gradient (e[0], e[1..3]),
// the gradient of I[lam_5 q_5] (e5), and I[div v] with its gradient (d).
// Eleven sums instead of the 28 of seven separate values and gradients.
__device__ __forceinline__ void gather_adj(const StencilD& s, const double* const (&q)[6],
                                           const double* __restrict__ div, const double (&lam)[6], int n,
                                           double (&e)[4], double (&e5)[3], double (&d)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) e[k] = d[k] = 0.0;
  e5[0] = e5[1] = e5[2] = 0.0;
  for_taps(s, n, [&](long long idx, double w, double wgx, double wgy, double wgz) {
    double c = lam[0] * q[0][idx];
#pragma unroll
    for (int k = 1; k < 5; ++k) c += lam[k] * q[k][idx];
    const double c5 = lam[5] * q[5][idx];
    const double dv = div[idx];
    e[0] += w * c;
    e[1] += wgx * c;
    e[2] += wgy * c;
    e[3] += wgz * c;
    e5[0] += wgx * c5;
    e5[1] += wgy * c5;
    e5[2] += wgz * c5;
    d[0] += w * dv;
    d[1] += wgx * dv;
    d[2] += wgy * dv;
    d[3] += wgz * dv;
  });
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

// One 16 x 4 x 4 brick of arrival voxels per 256-thread block (n >= 16, so the
// bricks tile the grid), bricks laid out x fastest, and consecutive block
// indices spread over the 8 XCDs so that each XCD sweeps a contiguous slab.
constexpr int kSlAdjBX = 16, kSlAdjBY = 4, kSlAdjBZ = 4;
constexpr int kSlAdjThreads = kSlAdjBX * kSlAdjBY * kSlAdjBZ;
static_assert(kSlAdjThreads == 256, "the tile helpers assume 256-thread blocks");
// LDS tile of the box of a brick's stencils, (16 + 3 + dx) x (4 + 3 + dy) x
// (4 + 3 + dz) nodes for a spread dx, dy, dz of its departure cells; 2048
// nodes cover a spread of 2 cells per axis.  A gather holds two FP64 values
// per node, the scatter two 64-bit fixed-point sums (the same 32 KiB).
constexpr int kSlAdjTile = 2048;

// Visit the 64 taps of a stencil in an LDS tile of G-value nodes whose
// origin is box and extent L: fn(vals, w, wgx, wgy, wgz).
template <int G, typename Fn>
__device__ __forceinline__ void tile_taps(const double* tile, const StencilD& s, const int (&box)[3],
                                          const int (&L)[3], Fn fn) {
  const int rx = s.ix - 1 - box[0], ry = s.iy - 1 - box[1], rz = s.iz - 1 - box[2];
#pragma unroll 1
  for (int r = 0; r < 16; ++r) {
    const int c = r >> 2, b = r & 3;
    const int base = ((rz + c) * L[1] + (ry + b)) * L[0] + rx;
    const double wz = pick4(s.wz, c), dz = pick4(s.dz, c), wy = pick4(s.wy, b), dy = pick4(s.dy, b);
    const double wzy = wz * wy, dzy = dz * wy, wzdy = wz * dy;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      double q[G];
      tile_get<G, double>(tile, base + a, q);
      fn(q, wzy * s.wx[a], wzy * s.dx[a], wzdy * s.wx[a], dzy * s.wx[a]);
    }
  }
}

// Stage the box of G fields into the tile (between barriers: the previous
// readers of the tile are done, and every thread sees the new contents).
template <int G>
__device__ __forceinline__ void tile_load(double* tile, const double* const (&src)[G], const int (&box)[3],
                                          const int (&L)[3], int n) {
  double sc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) sc[g] = 1.0;
  __syncthreads();
  tile_stage<double, G>(tile, src, sc, box[0], box[1], box[2], L, n);
  __syncthreads();
}

// Transposed interpolation of nf values per voxel at the stencil s: each
// tap's contribution w * val[f] goes to the node it was read from.  The
// values, targets and scales are in LDS (sval[f][thread], sout[f], sscale[f]).
// With the box in the tile (fits), contributions of two fields at a time
// are summed in LDS with integer atomics, then each tile node is added to
// global memory with one atomic per field; otherwise every contribution
// goes straight to a global atomic.  All sums are 64-bit fixed point, so
// both paths give the same integers.  Called by all threads of the block
// (block-uniform control flow).
__device__ void scatter_block(const Stencil& s, int f0, int nf, double (*sval)[kSlAdjThreads],
                              double* const* sout, const double* sscale, bool fits, const int (&box)[3],
                              const int (&L)[3], long long* tile, int n) {
  const int m = n - 1;
  if (!fits) {
    for (int f = f0; f < f0 + nf; ++f) {
      const double vf = sval[f][threadIdx.x], sc = sscale[f];
      double* const of = sout[f];
#pragma unroll 1
      for (int r = 0; r < 16; ++r) {
        const int c = r >> 2, b = r & 3;
        const long long yo = ((long long)((s.iz + c - 1) & m) * n + ((s.iy + b - 1) & m)) * n;
        const double wzy = pick4(s.wz, c) * pick4(s.wy, b) * vf;
#pragma unroll
        for (int a = 0; a < 4; ++a) fix_add(of + yo + ((s.ix + a - 1) & m), to_fix(wzy * s.wx[a], sc));
      }
    }
    return;
  }
  const int cnt = L[0] * L[1] * L[2];
  const int rx = s.ix - 1 - box[0], ry = s.iy - 1 - box[1], rz = s.iz - 1 - box[2];
  for (int f = f0; f < f0 + nf; f += 2) {
    const int g2 = (f + 1 < f0 + nf) ? 2 : 1;  // fields in this round (block-uniform)
    __syncthreads();  // the previous users of the tile are done
    for (int k = threadIdx.x; k < g2 * cnt; k += kSlAdjThreads) tile[k] = 0;
    __syncthreads();
    for (int g = 0; g < g2; ++g) {
      const double vf = sval[f + g][threadIdx.x], sc = sscale[f + g];
      long long* const tg = tile + g * cnt;
#pragma unroll 1
      for (int r = 0; r < 16; ++r) {
        const int c = r >> 2, b = r & 3;
        const double wzy = pick4(s.wz, c) * pick4(s.wy, b) * vf;
        const int row = ((rz + c) * L[1] + (ry + b)) * L[0] + rx;
#pragma unroll
        for (int a = 0; a < 4; ++a)
          atomicAdd(reinterpret_cast<unsigned long long*>(&tg[row + a]),
                    static_cast<unsigned long long>(to_fix(wzy * s.wx[a], sc)));
      }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < g2 * cnt; k += kSlAdjThreads) {
      const long long t = tile[k];
      if (t != 0) {
        const int g = k >= cnt ? 1 : 0;
        const int e = k - g * cnt;
        const int tx = e % L[0], ty = (e / L[0]) % L[1], tz = e / (L[0] * L[1]);
        const long long idx =
            ((long long)((box[2] + tz) & m) * n + ((box[1] + ty) & m)) * n + ((box[0] + tx) & m);
        fix_add(sout[f + g] + idx, t);
      }
    }
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

// Transpose of the semi-Lagrangian step (Sec. 3) for one arrival voxel per
// thread.  With X* = x - s v, v* = I[v](X*), X = x - s/2 (v + v*) and the
// Heun factor cfac = 1 - dt/2 (div(X) + div(x)) + dt^2/2 div(X) div(x), the
// forward step is q+_k(x) = cfac I[q_k](X) for k < 5 and q+_5 = I[q_5](X).
// The gathers at X* and X read LDS halo tiles of the brick's stencil box (or
// global memory when the box exceeds the tile); the transposed
// interpolations accumulate in the same tiles.  Interpolation weights are
// recomputed from the departure points where they are needed, rather than
// held across the gathers and scatters, so that the kernel stays within the
// register file.
__global__ void __launch_bounds__(kSlAdjThreads) k_sl_adj(SLAdjArgs a, const GradScalars* gs) {
  __shared__ __align__(16) long long tile[2 * kSlAdjTile];
  __shared__ double sval[10][kSlAdjThreads];
  __shared__ double* sout[10];
  __shared__ double sscale[10];
  __shared__ int red[24];
  double* const dtile = reinterpret_cast<double*>(tile);
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
  // X*, computed once: the scatter's stencil must have the gather's floors
  const double XS[3] = {jx - s * vx, jy - s * vy, jz - s * vz};
  int box1[3], L1[3], box2[3], L2[3];
  bool fits1, fits2;
  // v* = I[v](X*) and its gradient gv[b][c] = d/dj_c I[v_b](X*)
  double vs[3], gv[3][3];
#pragma unroll
  for (int b = 0; b < 3; ++b) vs[b] = gv[b][0] = gv[b][1] = gv[b][2] = 0.0;
  {
    StencilD st;
    st.set(XS[0], XS[1], XS[2]);
    int lo[3] = {st.ix, st.iy, st.iz}, hi[3] = {st.ix, st.iy, st.iz};
    block_box(lo, hi, red);
    fits1 = box_fits(lo, hi, n, kSlAdjTile, box1, L1);
    if (fits1) {
      const double* const s01[2] = {a.vx, a.vy};
      tile_load<2>(dtile, s01, box1, L1, n);
      tile_taps<2>(dtile, st, box1, L1, [&](const double (&q)[2], double w, double wgx, double wgy, double wgz) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          vs[b] += w * q[b];
          gv[b][0] += wgx * q[b];
          gv[b][1] += wgy * q[b];
          gv[b][2] += wgz * q[b];
        }
      });
      const double* const s2[1] = {a.vz};
      tile_load<1>(dtile, s2, box1, L1, n);
      tile_taps<1>(dtile, st, box1, L1, [&](const double (&q)[1], double w, double wgx, double wgy, double wgz) {
        vs[2] += w * q[0];
        gv[2][0] += wgx * q[0];
        gv[2][1] += wgy * q[0];
        gv[2][2] += wgz * q[0];
      });
    } else {
      gather_vel(st, a.vx, a.vy, a.vz, n, vs, gv);
    }
  }
  const double X[3] = {jx - 0.5 * s * (vx + vs[0]), jy - 0.5 * s * (vy + vs[1]), jz - 0.5 * s * (vz + vs[2])};
  double lam[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) lam[k] = a.lam[k][v];
  // at X: e = I[sum_{k<5} lam_k q_k] with its gradient, grad I[lam_5 q_5], I[div v] with its gradient
  double e[4], e5[3], dq[4];
  {
    StencilD st;
    st.set(X[0], X[1], X[2]);
    int lo[3] = {st.ix, st.iy, st.iz}, hi[3] = {st.ix, st.iy, st.iz};
    block_box(lo, hi, red);
    fits2 = box_fits(lo, hi, n, kSlAdjTile, box2, L2);
    if (fits2) {
#pragma unroll
      for (int k = 0; k < 4; ++k) e[k] = dq[k] = 0.0;
      e5[0] = e5[1] = e5[2] = 0.0;
      auto acc_e = [&](double c, double w, double wgx, double wgy, double wgz) {
        e[0] += w * c;
        e[1] += wgx * c;
        e[2] += wgy * c;
        e[3] += wgz * c;
      };
      const double* const p01[2] = {a.q[0], a.q[1]};
      tile_load<2>(dtile, p01, box2, L2, n);
      tile_taps<2>(dtile, st, box2, L2, [&](const double (&q)[2], double w, double wgx, double wgy, double wgz) {
        acc_e(lam[0] * q[0] + lam[1] * q[1], w, wgx, wgy, wgz);
      });
      const double* const p23[2] = {a.q[2], a.q[3]};
      tile_load<2>(dtile, p23, box2, L2, n);
      tile_taps<2>(dtile, st, box2, L2, [&](const double (&q)[2], double w, double wgx, double wgy, double wgz) {
        acc_e(lam[2] * q[0] + lam[3] * q[1], w, wgx, wgy, wgz);
      });
      const double* const p45[2] = {a.q[4], a.q[5]};
      tile_load<2>(dtile, p45, box2, L2, n);
      tile_taps<2>(dtile, st, box2, L2, [&](const double (&q)[2], double w, double wgx, double wgy, double wgz) {
        acc_e(lam[4] * q[0], w, wgx, wgy, wgz);
        const double c5 = lam[5] * q[1];
        e5[0] += wgx * c5;
        e5[1] += wgy * c5;
        e5[2] += wgz * c5;
      });
      const double* const pd[1] = {a.div};
      tile_load<1>(dtile, pd, box2, L2, n);
      tile_taps<1>(dtile, st, box2, L2, [&](const double (&q)[1], double w, double wgx, double wgy, double wgz) {
        dq[0] += w * q[0];
        dq[1] += wgx * q[0];
        dq[2] += wgy * q[0];
        dq[3] += wgz * q[0];
      });
    } else {
      gather_adj(st, a.q, a.div, lam, n, e, e5, dq);
    }
  }
  const double dX = dq[0];
  const double cfac = 1.0 - 0.5 * dt * (dX + d0) + 0.5 * dt * dt * dX * d0;
  const double cbar = e[0];  // sum_{k<5} lam_k I[q_k](X)
  const double bar6 = cbar * (-0.5 * dt + 0.5 * dt * dt * d0);
  const double ddirect = cbar * (-0.5 * dt + 0.5 * dt * dt * dX);
  // adjoint of X: sum_k bar_k grad I[q_k](X), bar_6 belonging to div v
  double vsb[3], vown[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) vsb[c] = -0.5 * s * (cfac * e[1 + c] + e5[c] + bar6 * dq[1 + c]);
  // X* moves with v (directly) and through v*
#pragma unroll
  for (int c = 0; c < 3; ++c) vown[c] = vsb[c] - s * (vsb[0] * gv[0][c] + vsb[1] * gv[1][c] + vsb[2] * gv[2][c]);
  // values, targets and fixed-point scales of the ten scattered fields
#pragma unroll
  for (int k = 0; k < 5; ++k) sval[k][threadIdx.x] = lam[k] * cfac;
  sval[5][threadIdx.x] = lam[5];
  sval[6][threadIdx.x] = bar6;
#pragma unroll
  for (int c = 0; c < 3; ++c) sval[7 + c][threadIdx.x] = vsb[c];
  if (threadIdx.x == 0) {
    double scale[10];
    bool finite;
    sl_adj_scales(gs, dt, s, scale, finite);
    double* const t[10] = {a.out[0], a.out[1], a.out[2], a.out[3], a.out[4], a.out[5], a.divb,
                           a.vb[0], a.vb[1], a.vb[2]};
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      sout[k] = t[k];
      sscale[k] = scale[k];
    }
  }
  __syncthreads();
  {
    double xx = X[0], xy = X[1], xz = X[2];
    asm volatile("" : "+v"(xx), "+v"(xy), "+v"(xz));
    Stencil st;
    st.set(xx, xy, xz);
    scatter_block(st, 0, 7, sval, sout, sscale, fits2, box2, L2, tile, n);
  }
  fix_add(a.divb + v, to_fix(ddirect, sscale[6]));
  {
    // X* again, opaque to the compiler, which would otherwise keep the
    // weights of the first gather alive across the second
    double xs = XS[0], ys = XS[1], zs = XS[2];
    asm volatile("" : "+v"(xs), "+v"(ys), "+v"(zs));
    Stencil st;
    st.set(xs, ys, zs);
    scatter_block(st, 7, 3, sval, sout, sscale, fits1, box1, L1, tile, n);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) fix_add(a.vb[c] + v, to_fix(vown[c], sscale[7 + c]));
}

// ------------------------------------------------------ initial condition
// part[k * nb + block] = sum over the block's voxels of phi_k * lam_p, for
// the kIcGroup seeds k of grid row blockIdx.y: lam_p is read once per group
// of seeds, and each seed's sum runs in the same order as alone.
constexpr int kIcGroup = 16;
__global__ void __launch_bounds__(256) k_ic_adj(int n, const double* ic, int n_ic, const double* lam_p,
                                                double* part) {
  const long long V = (long long)n * n * n;
  const int k0 = blockIdx.y * kIcGroup;
  const int ng = min(kIcGroup, n_ic - k0);  // block-uniform
  const double h = 2.0 * M_PI / n, twopi = 2.0 * M_PI;
  double acc[kIcGroup];
#pragma unroll
  for (int g = 0; g < kIcGroup; ++g) acc[g] = 0.0;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < V;
       v += (long long)gridDim.x * blockDim.x) {
    const int jx = (int)(v % n), jy = (int)((v / n) % n), jz = (int)(v / ((long long)n * n));
    const double lp = lam_p[v];
#pragma unroll
    for (int g = 0; g < kIcGroup; ++g) {
      if (g < ng) {
        const double* c = ic + 5 * (k0 + g);
        double dx = h * jx - c[0], dy = h * jy - c[1], dz = h * jz - c[2];
        dx -= twopi * rint(dx / twopi);
        dy -= twopi * rint(dy / twopi);
        dz -= twopi * rint(dz / twopi);
        const double d2 = dz * dz + dy * dy + dx * dx;
        acc[g] += exp(-d2 / (2.0 * c[3] * c[3])) * lp;
      }
    }
  }
  __shared__ double sh[kIcGroup][4];
#pragma unroll
  for (int g = 0; g < kIcGroup; ++g) {
    const double s = wave_sum_d(acc[g]);
    if ((threadIdx.x & 63) == 0) sh[g][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  const int g = threadIdx.x;
  if (g < ng) part[(long long)(k0 + g) * gridDim.x + blockIdx.x] = sh[g][0] + sh[g][1] + sh[g][2] + sh[g][3];
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
  hipLaunchKernelGGL(k_ic_adj, dim3(nb, (n_ic + kIcGroup - 1) / kIcGroup), dim3(256), 0, st, n, ic, n_ic, lam_p,
                     part);
  hipLaunchKernelGGL(k_ic_adj_sum, dim3((n_ic + 63) / 64), dim3(64), 0, st, part, nb, n_ic, out);
}

}  // namespace tumor
