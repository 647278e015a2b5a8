// Pointwise, semi-Lagrangian and Krylov-vector kernels for gfx950.
//
// Reductions are deterministic: each block writes one partial per quantity,
// and a one-block kernel queued right after sums the partials in a fixed order
// and publishes the result to device scalars that later kernels and the host
// read.  The grid size of a reduction kernel is a fixed function of the
// problem size, so results do not depend on timing.
#include <algorithm>
#include <climits>
#include <cmath>

#include "kernels.hpp"
#include "prec.hpp"
#include "sl_tile.hpp"

namespace tumor {

// ------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-reduce v[] and store this block's partials (plain stores, no fence):
// a one-block finishing kernel launched next totals them, the kernel boundary
// making them visible.  A device-scope fence per block would instead push the
// block's whole output out of its XCD's L2.
template <int NV>
__device__ void block_store_partials(double (&v)[NV], double* part) {
  __shared__ double sh[NV][kRedThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double s = wave_sum(v[i]);
    if (lane == 0) sh[i][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < kRedThreads / 64; ++w) s += sh[i][w];
      part[(long long)blockIdx.x * kPartialsPerBlock + i] = s;
    }
  }
}

// Fixed-order totals of NV partials of nb blocks (one block of kRedThreads).
template <int NV>
__device__ void total_partials(double (&tot)[NV], const double* part, int nb, int stride) {
  __shared__ double sh[NV][kRedThreads / 64];
  double v[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = 0.0;
  for (int b = threadIdx.x; b < nb; b += kRedThreads) {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] += part[(long long)b * stride + i];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double s = wave_sum(v[i]);
    if (lane == 0) sh[i][wv] = s;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
    for (int w = 0; w < kRedThreads / 64; ++w) s += sh[i][w];
    tot[i] = s;
  }
}

static inline int red_blocks(long long count) {
  long long b = (count + kRedThreads - 1) / kRedThreads;
  if (b > kRedBlocksMax) b = kRedBlocksMax;
  if (b < 1) b = 1;
  return (int)b;
}

// ------------------------------------------------------ reaction + refresh
// Smoothed Heaviside (1 + tanh(x/eps))/2 in its cancellation-free form
// 1/(1 + exp(-2x/eps)); exp overflow gives exactly 0.
__device__ __forceinline__ double heav(double x, double eps) { return 1.0 / (1.0 + exp(-2.0 * x / eps)); }

__device__ __forceinline__ double logistic_flow(double y, double r, double t) {
  const double e = exp(r * t);
  return y * e / (1.0 + y * (e - 1.0));
}

__global__ void __launch_bounds__(kRedThreads) k_react(ReactArgs a) {
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  const ReactConsts& rc = a.rc;
  const RefreshConsts& fc = a.fc;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < a.V; v += stride) {
    double p = a.p[v], n = a.n[v], g = a.g[v], w = a.w[v], o = a.o[v], l = a.l[v], f = a.f[v];
    double i = a.i_dd[v];
    if (a.do_reaction && a.single) {
      // Single-species model (e:rd): logistic growth rho c (1 - c) with the
      // frozen rho (e:reac_op, e:reaction_op), exact over dt; g and w lose the
      // diffusion and growth increments in proportion g : w (e:gm, e:wm).
      const double c_dag = a.i_dag[v], c_dd = i;
      const double dR = logistic_flow(c_dd, a.rho[v], rc.dt) - c_dd;
      const double c1 = c_dd + dR;
      const double s = (c_dd - c_dag) + dR;
      const double gw = g + w;
      const bool small = gw < 1e-12;
      const double phig = small ? 0.5 : g / gw;
      const double phiw = small ? 0.5 : w / gw;
      p = c1;
      i = 0.0;
      g = g - phig * s;
      w = w - phiw * s;
      a.po[v] = p; a.io[v] = i; a.no[v] = n; a.go[v] = g; a.wo[v] = w; a.oo[v] = o; a.lo[v] = l;
      a.fo[v] = f;
    } else if (a.do_reaction) {
      const double dt = rc.dt;
      const double dD = i - a.i_dag[v];
      const double rho_p = a.rho[v];
      const double rho_i = rc.rho_inv_frac * rho_p;
      const double alpha = rc.alpha0 * heav(rc.o_inv - o, rc.eps);
      const double beta = rc.beta0 * heav(rc.sigma_b - p - i, rc.eps) * o;
      const double h = rc.gamma * heav(rc.o_hyp - o, rc.eps);
      double kap = (o - rc.o_mit) / (rc.o_inv - rc.o_mit);
      kap = kap < 0.0 ? 0.0 : (kap > 1.0 ? 1.0 : kap);
      const double dRp = logistic_flow(p, rho_p * kap, dt) - p;
      const double dRi = logistic_flow(i, rho_i * kap, dt) - i;
      const double p1 = p + dRp + dt * (-alpha * p + beta * i - h * p);
      const double i1 = i + dRi + dt * (alpha * p - beta * i - h * i);
      const double n1 = n + dt * h * (p + i + g + w);
      const double s = dD + dRp + dRi;
      const double gw = g + w;
      const bool small = gw < 1e-12;
      const double phig = small ? 0.5 : g / gw;
      const double phiw = small ? 0.5 : w / gw;
      const double g1 = g - phig * s - dt * h * g;
      const double w1 = w - phiw * s - dt * h * w;
      const double o1 = o + dt * (-rc.delta_p * p1 + rc.delta_s * (rc.o_heal - o) * (g1 + w1));
      double l1 = l;
      if (rc.edema) l1 = l + dt * (rc.delta_e * i1 / (i1 + rc.delta_half) * (1.0 - i1) - rc.delta_l * l);
      p = p1; i = i1; n = n1; g = g1; w = w1; o = o1; l = l1;
      a.po[v] = p; a.io[v] = i; a.no[v] = n; a.go[v] = g; a.wo[v] = w; a.oo[v] = o; a.lo[v] = l;
      a.fo[v] = f;
    }
    // refresh
    const double tau = p + i + n;
    const double K = fc.k_w * w + fc.k_g * g + fc.k_f * f;
    const double rho = fc.rho_w * w + fc.rho_g * g;
    const double b = a.bg[v];
    const double mu = fc.mu_w * w + fc.mu_g * g + fc.mu_f * f + fc.mu_t * tau + fc.mu_b * b;
    const double lam = fc.la_w * w + fc.la_g * g + fc.la_f * f + fc.la_t * tau + fc.la_b * b;
    const double eta = fc.eta_t * tau + fc.eta_h * (g + w + f) + fc.eta_b * b;
    a.K[v] = K; a.rho[v] = rho; a.mu[v] = mu; a.lam[v] = lam; a.eta[v] = eta;
    if (a.K32) {
      a.K32[v] = (float)K; a.mu32[v] = (float)mu; a.lam32[v] = (float)lam; a.eta32[v] = (float)eta;
    }
    acc[0] += K; acc[1] += mu; acc[2] += lam; acc[3] += eta;
    acc[4] += p; acc[5] += i; acc[6] += n; acc[7] += o; acc[8] += l; acc[9] += g; acc[10] += w;
    acc[11] += f;
  }
  block_store_partials<12>(acc, a.partials);
}

// ------------------------------------------------- one-block finishing kernels
// Each totals the block partials of the kernel queued just before it (fixed
// order) and publishes the scalars.
__global__ void __launch_bounds__(kRedThreads) k_fin_react(CoefScalars* cs, const double* part, int nb, long long V) {
  double tot[12];
  total_partials<12>(tot, part, nb, kPartialsPerBlock);
  if (threadIdx.x == 0) {
    const double iv = 1.0 / (double)V;
    cs->Kbar = tot[0] * iv;
    cs->mubar = tot[1] * iv;
    cs->lambar = tot[2] * iv;
    cs->etabar = tot[3] * iv;
    int bad = 0;
    for (int k = 0; k < 8; ++k) {
      cs->mass[k] = tot[4 + k];
      if (!isfinite(tot[4 + k])) bad = 1;
    }
    cs->bad = bad;
  }
}

// ||b||^2 and ||r||^2 of a fresh residual; resets the solve state.
__global__ void __launch_bounds__(kRedThreads) k_fin_resid(SolveScalars* sv, const double* part, int nb) {
  double tot[2];
  total_partials<2>(tot, part, nb, kPartialsPerBlock);
  if (threadIdx.x == 0) {
    sv->bb = tot[0];
    sv->rr = tot[1];
    sv->it = 0;
    sv->done = 0;
    sv->conv = 0;
    sv->bad = (isfinite(tot[0]) && isfinite(tot[1])) ? 0 : 1;
  }
}

// rho = <r, M^-1 r> at the start of a PCG solve.
__global__ void __launch_bounds__(kRedThreads) k_fin_start(SolveScalars* sv, const double* part, int nb) {
  double tot[1];
  total_partials<1>(tot, part, nb, kPartialsPerBlock);
  if (threadIdx.x == 0) {
    sv->rho = tot[0];
    sv->it = 0;
    sv->conv = 0;
    const bool ok = isfinite(tot[0]) && tot[0] > 0.0;
    sv->bad = ok ? 0 : 1;
    sv->done = ok ? 0 : 1;
  }
}

// ----------------------------------------------------------- diagnostics
// Per-block slots: 0 max |u|^2 / h^2, 1 max(-tr T), 2 max tr T, 3 max tau,
// 4 max(-J), 5 max J, 6 sum (J - 1)^2, 7 max squared seed distance of the
// points displaced by >= thr voxels (-1: none).  Slot 6 sums, the others take
// maxima.
constexpr int kDiagSlots = 8;

__device__ __forceinline__ double diag_combine(int k, double a, double b) { return k == 6 ? a + b : fmax(a, b); }

__global__ void __launch_bounds__(kRedThreads) k_diag(DiagArgs a) {
  const int n = a.n;
  const long long V = (long long)n * n * n;
  const double L = 2.0 * M_PI;
  double acc[kDiagSlots];
#pragma unroll
  for (int k = 0; k < kDiagSlots; ++k) acc[k] = (k == 6) ? 0.0 : -INFINITY;
  for (long long v = (long long)blockIdx.x * kRedThreads + threadIdx.x; v < V;
       v += (long long)gridDim.x * kRedThreads) {
    double F[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) F[i][j] = a.f[3 + 3 * j + i][v];
    const double mu = a.mu[v], lam = a.lam[v];
    const double tr = F[0][0] + F[1][1] + F[2][2];
    const double Txx = mu * (F[0][0] + F[0][0]) + lam * tr;
    const double Tyy = mu * (F[1][1] + F[1][1]) + lam * tr;
    const double Tzz = mu * (F[2][2] + F[2][2]) + lam * tr;
    const double Txy = mu * (F[0][1] + F[1][0]);
    const double trace = Txx + Tyy + Tzz;
    const double hx = 0.5 * (Txx - Tyy);
    const double tau = sqrt(hx * hx + Txy * Txy);
    const double a00 = F[0][0] + 1.0, a11 = F[1][1] + 1.0, a22 = F[2][2] + 1.0;
    const double J = a00 * (a11 * a22 - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * a22 - F[1][2] * F[2][0]) +
                     F[0][2] * (F[1][0] * F[2][1] - a11 * F[2][0]);
    if (a.trace) a.trace[v] = trace;
    if (a.shear) a.shear[v] = tau;
    if (a.jac) a.jac[v] = J;
    const double ux = a.f[0][v], uy = a.f[1][v], uz = a.f[2][v];
    const double umag = sqrt(ux * ux + uy * uy + uz * uz) / a.h;
    acc[0] = fmax(acc[0], umag);
    acc[1] = fmax(acc[1], -trace);
    acc[2] = fmax(acc[2], trace);
    acc[3] = fmax(acc[3], tau);
    acc[4] = fmax(acc[4], -J);
    acc[5] = fmax(acc[5], J);
    acc[6] += (J - 1.0) * (J - 1.0);
    if (a.n_ic > 0 && umag >= a.thr) {
      const int jx = (int)(v % n), jy = (int)((v / n) % n), jz = (int)(v / ((long long)n * n));
      const double q[3] = {a.h * jx, a.h * jy, a.h * jz};
      double best = INFINITY;
      for (int k = 0; k < a.n_ic; ++k) {
        double d2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double d = q[c] - a.ic[5 * k + c];
          d = d - L * rint(d / L);
          d2 = d2 + d * d;
        }
        best = fmin(best, d2);
      }
      acc[7] = fmax(acc[7], best);
    }
  }
  __shared__ double sh[kDiagSlots][kRedThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kDiagSlots; ++k) {
    double t = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t = diag_combine(k, t, __shfl_xor(t, off, 64));
    if (lane == 0) sh[k][wv] = t;
  }
  __syncthreads();
  if (threadIdx.x < kDiagSlots) {
    const int k = threadIdx.x;
    double t = sh[k][0];
    for (int w = 1; w < kRedThreads / 64; ++w) t = diag_combine(k, t, sh[k][w]);
    a.partials[(long long)blockIdx.x * kPartialsPerBlock + k] = t;
  }
}

__global__ void __launch_bounds__(kRedThreads) k_fin_diag(const double* part, int nb, double h, double* res) {
  __shared__ double sh[kDiagSlots][kRedThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kDiagSlots; ++k) {
    double t = (k == 6) ? 0.0 : -INFINITY;
    for (int b = threadIdx.x; b < nb; b += kRedThreads) t = diag_combine(k, t, part[(long long)b * kPartialsPerBlock + k]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t = diag_combine(k, t, __shfl_xor(t, off, 64));
    if (lane == 0) sh[k][wv] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[kDiagSlots];
    for (int k = 0; k < kDiagSlots; ++k) {
      t[k] = sh[k][0];
      for (int w = 1; w < kRedThreads / 64; ++w) t[k] = diag_combine(k, t[k], sh[k][w]);
    }
    res[0] = t[0];
    res[1] = -t[1];
    res[2] = t[2];
    res[3] = t[3];
    res[4] = -t[4];
    res[5] = t[5];
    res[6] = sqrt(h * h * h * t[6]);
    res[7] = t[7] >= 0.0 ? sqrt(t[7]) / h : 0.0;
  }
}

void launch_diag(const DiagArgs& a, double* results, hipStream_t st) {
  const int nb = red_blocks((long long)a.n * a.n * a.n);
  hipLaunchKernelGGL(k_diag, dim3(nb), dim3(kRedThreads), 0, st, a);
  hipLaunchKernelGGL(k_fin_diag, dim3(1), dim3(kRedThreads), 0, st, a.partials, nb, a.h, results);
}

void launch_react(const ReactArgs& a, hipStream_t st) {
  const int nb = red_blocks(a.V);
  hipLaunchKernelGGL(k_react, dim3(nb), dim3(kRedThreads), 0, st, a);
  hipLaunchKernelGGL(k_fin_react, dim3(1), dim3(kRedThreads), 0, st, a.cs, a.partials, nb, a.V);
}

// ------------------------------------------------------- initial condition
__global__ void k_ic(int n, const double* __restrict__ ic, int n_ic, double* __restrict__ p0) {
  const long long V = (long long)n * n * n;
  const double h = 2.0 * M_PI / n;
  const double twopi = 2.0 * M_PI;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < V;
       v += (long long)gridDim.x * blockDim.x) {
    const int jx = (int)(v % n), jy = (int)((v / n) % n), jz = (int)(v / ((long long)n * n));
    const double x = h * jx, y = h * jy, z = h * jz;
    double s = 0.0;
    for (int k = 0; k < n_ic; ++k) {
      const double* c = ic + 5 * k;
      double dx = x - c[0], dy = y - c[1], dz = z - c[2];
      dx -= twopi * rint(dx / twopi);
      dy -= twopi * rint(dy / twopi);
      dz -= twopi * rint(dz / twopi);
      const double d2 = dz * dz + dy * dy + dx * dx;
      s += c[4] * exp(-d2 / (2.0 * c[3] * c[3]));
    }
    p0[v] = s;
  }
}

__global__ void k_fill(double* __restrict__ p, double value, long long count) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < count;
       v += (long long)gridDim.x * blockDim.x)
    p[v] = value;
}

void launch_fill(double* p, double value, long long count, hipStream_t st) {
  long long blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks > 0) hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, p, value, count);
}

// Streaming copy, one 16-byte vector per thread and no loop: the launch shape
// that reads and writes HBM fastest on this part (a bandwidth reference for the
// other kernels' rates).
__global__ void k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, long long count) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i];
}

void launch_stream_copy(const void* src, void* dst, long long bytes, hipStream_t st) {
  const long long count = bytes / 16;
  const long long blocks = (count + 255) / 256;
  if (blocks > 0)
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<const uint4*>(src),
                       static_cast<uint4*>(dst), count);
}

void launch_ic(int n, const double* ic, int n_ic, double* p0, hipStream_t st) {
  const long long V = (long long)n * n * n;
  long long blocks = (V + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_ic, dim3((unsigned)blocks), dim3(256), 0, st, n, ic, n_ic, p0);
}

// --------------------------------------------------------- semi-Lagrangian
template <typename RC>
__device__ __forceinline__ void lagrange4(RC t, RC (&w)[4]) {
  w[0] = -t * (t - RC(1)) * (t - RC(2)) / RC(6);
  w[1] = (t + RC(1)) * (t - RC(1)) * (t - RC(2)) / RC(2);
  w[2] = -(t + RC(1)) * t * (t - RC(2)) / RC(2);
  w[3] = (t + RC(1)) * t * (t - RC(1)) / RC(6);
}

// Tricubic Lagrange interpolation of NF periodic fields at one point
// (grid-index coordinates, computed in FP64; weights and sums in RC).
template <typename RC, int NF>
__device__ __forceinline__ void interp_pt(const double* const (&q)[NF], double jx, double jy, double jz, int n,
                                          RC (&out)[NF]) {
  const double bx = floor(jx), by = floor(jy), bz = floor(jz);
  RC wx[4], wy[4], wz[4];
  lagrange4<RC>(RC(jx - bx), wx);
  lagrange4<RC>(RC(jy - by), wy);
  lagrange4<RC>(RC(jz - bz), wz);
  const int ix = (int)(long long)bx, iy = (int)(long long)by, iz = (int)(long long)bz;
  const int m = n - 1;
#pragma unroll
  for (int f = 0; f < NF; ++f) out[f] = RC(0);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const long long zo = (long long)((iz + c - 1) & m) * n * n;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const long long yo = zo + (long long)((iy + b - 1) & m) * n;
      const RC wzy = wz[c] * wy[b];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const long long idx = yo + ((ix + a - 1) & m);
        const RC wt = wzy * wx[a];
#pragma unroll
        for (int f = 0; f < NF; ++f) out[f] += wt * RC(q[f][idx]);
      }
    }
  }
}

// Power-of-two scale 2^-e that brings max |q| = m to [1, 2) (1 for m = 0 or
// a non-finite m).  Multiplying by it is exact, so a field can be rounded to
// FP32 after scaling without leaving FP32's normal range, and unscaled in FP64.
__device__ __forceinline__ double pow2_scale(unsigned long long bits) {
  const double m = __longlong_as_double((long long)bits);
  return (m > 0.0 && m < INFINITY) ? ldexp(1.0, -ilogb(m)) : 1.0;
}

// max |q| of the six transported fields (mixed precision): block maxima,
// combined by atomic max on the bits of the non-negative doubles.
__global__ void __launch_bounds__(256) k_sl_scan(SLArgs a, CoefScalars* cs) {
  const double* const q[6] = {a.p, a.i, a.n, a.g, a.w, a.f};
  const long long V = (long long)a.n_grid * a.n_grid * a.n_grid;
  double m[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < V; v += (long long)gridDim.x * 256) {
#pragma unroll
    for (int f = 0; f < 6; ++f) m[f] = fmax(m[f], fabs(q[f][v]));
  }
  __shared__ double sh[6][4];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    double t = m[f];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t = fmax(t, __shfl_xor(t, off, 64));
    if ((threadIdx.x & 63) == 0) sh[f][threadIdx.x >> 6] = t;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int f = threadIdx.x;
    const double t = fmax(fmax(sh[f][0], sh[f][1]), fmax(sh[f][2], sh[f][3]));
    atomicMax(&cs->qmax_bits[f], (unsigned long long)__double_as_longlong(t));
  }
}

// max over a 256-thread block of c, combined into cs->cfl_bits.
__device__ __forceinline__ void block_max_cfl(double c, CoefScalars* cs) {
  if (!(c >= 0.0)) c = INFINITY;  // a NaN velocity reports an infinite CFL number
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c = fmax(c, __shfl_xor(c, off, 64));
  __shared__ double sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    atomicMax(&cs->cfl_bits, (unsigned long long)__double_as_longlong(m));
  }
}

// ------------------------------------------- LDS-tiled semi-Lagrangian step
// Semi-Lagrangian step of the transported fields (Sec. 3): RK2
// characteristics X* = x - dt v(x), X = x - dt/2 (v(x) + v(X*)), tricubic
// values at X, and Heun's method for the conservative source
// g(nu, x) = -nu div v(x) of p, i, n, g, w; f is transported without source.
//
// One 256-thread block takes a BX x BY x BZ brick of arrival voxels (VPT per
// thread, a thread's voxels 256 / (BX BY) planes apart in z).  For each of the
// two gather stages (v at X*, then p, i, n, g, w, f and div v at X) the block
// reduces the floors of its departure points to their bounding box, widens it
// by the stencil reach (-1 .. +2), copies that box of the needed fields from
// HBM into LDS once (coalesced rows, periodic wrap), and every voxel then
// reads its 64 taps from the tile: G values per 16-byte LDS node, several
// passes per stage.  A box larger than the tile (departure points of one
// brick spread wider than the tile holds) makes that stage of that block
// gather from global memory instead, with the same arithmetic.
//
// Interpolation type RC: FP64, or FP32 in the mixed precision.  In FP32 each
// transported field is multiplied by the power of two that brings its
// maximum |q| to [1, 2) before rounding (exact), and the result is unscaled in
// FP64: the interpolation and the Heun update are linear in q, so the scaling
// changes no result while fields far below FP32's normal range (the necrotic
// cells early on) keep FP32's relative precision instead of flushing to zero.
// Departure points and the stencil weights' arguments stay FP64.  Within a
// voxel the tap order (z, then y, then x; weight wz wy, then times wx) is
// fixed, so every path gives the same bits.

// Stencil of one point: base node floor(X) - 1 per axis and the weights.
template <typename RC>
struct Stencil {
  int ix, iy, iz;  // floor of the point (unwrapped grid index)
  RC wx[4], wy[4], wz[4];
  __device__ __forceinline__ void set(double jx, double jy, double jz) {
    const double bx = floor(jx), by = floor(jy), bz = floor(jz);
    lagrange4<RC>(RC(jx - bx), wx);
    lagrange4<RC>(RC(jy - by), wy);
    lagrange4<RC>(RC(jz - bz), wz);
    ix = (int)(long long)bx;
    iy = (int)(long long)by;
    iz = (int)(long long)bz;
  }
};

// out[0..G) += tricubic sum over the tile.
template <typename RC, int G>
__device__ __forceinline__ void tile_gather(const RC* tile, const Stencil<RC>& st, int x0, int y0, int z0,
                                            const int (&L)[3], RC* out) {
  const int rx = st.ix - 1 - x0, ry = st.iy - 1 - y0, rz = st.iz - 1 - z0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int base = ((rz + c) * L[1] + (ry + b)) * L[0] + rx;
      const RC wzy = st.wz[c] * st.wy[b];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const RC wt = wzy * st.wx[a];
        RC val[G];
        tile_get<G, RC>(tile, base + a, val);
#pragma unroll
        for (int g = 0; g < G; ++g) out[g] += wt * val[g];
      }
    }
  }
}

// The same sum from the global FP64 fields (fallback for an oversized box).
template <typename RC, int G>
__device__ __forceinline__ void global_gather(const double* const (&src)[G], const double (&sc)[G],
                                              const Stencil<RC>& st, int n, RC* out) {
  const int m = n - 1;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const long long zo = (long long)((st.iz + c - 1) & m) * n * n;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const long long yo = zo + (long long)((st.iy + b - 1) & m) * n;
      const RC wzy = st.wz[c] * st.wy[b];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const long long idx = yo + ((st.ix + a - 1) & m);
        const RC wt = wzy * st.wx[a];
#pragma unroll
        for (int g = 0; g < G; ++g)
          if (src[g]) out[g] += wt * RC(sc[g] * src[g][idx]);
      }
    }
  }
}

// One gather pass of G fields for all voxels of the thread.
template <typename RC, int G, int VPT>
__device__ __forceinline__ void sl_pass(RC* tile, bool fits, const double* const (&src)[G], const double (&sc)[G],
                                        const int (&box)[3], const int (&L)[3], const Stencil<RC> (&st)[VPT],
                                        int n, RC (&acc)[VPT][8], int slot) {
  if (fits) {
    __syncthreads();  // the previous pass has finished reading the tile
    tile_stage<RC, G>(tile, src, sc, box[0], box[1], box[2], L, n);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < VPT; ++k) tile_gather<RC, G>(tile, st[k], box[0], box[1], box[2], L, &acc[k][slot]);
  } else {
#pragma unroll
    for (int k = 0; k < VPT; ++k) global_gather<RC, G>(src, sc, st[k], n, &acc[k][slot]);
  }
}

template <typename RC, int BX, int BY, int BZ, int CAP>
__global__ void __launch_bounds__(256) k_sl_tile(SLArgs a, CoefScalars* cs) {
  constexpr int ZS = 256 / (BX * BY);        // z distance of a thread's voxels
  constexpr int VPT = BZ / ZS;
  static_assert(256 % (BX * BY) == 0 && BZ % ZS == 0, "brick shape");
  constexpr int GV = sizeof(RC) == 4 ? 4 : 2;  // values per 16-byte LDS node
  __shared__ __align__(16) RC tile[CAP * (16 / sizeof(RC))];   // CAP 16-byte nodes
  __shared__ int red[24];
  const int n = a.n_grid;
  // bricks: x fastest, then z in groups of 4, then y; blocks dealt to the
  // eight XCDs in turn, each XCD sweeping a contiguous slab of bricks
  const unsigned nb = gridDim.x;
  const unsigned id = (blockIdx.x & 7u) * (nb >> 3) + (blockIdx.x >> 3);
  const unsigned nbx = (unsigned)n / BX, nby = (unsigned)n / BY;
  const unsigned bx = id % nbx;
  unsigned r = id / nbx;
  const unsigned zl = r & 3u;
  r >>= 2;
  const unsigned by = r % nby, zg = r / nby;
  const int t = threadIdx.x;
  const int jx = (int)(bx * BX) + (t % BX);
  const int jy = (int)(by * BY) + ((t / BX) % BY);
  const int jz0 = (int)((zg * 4 + zl) * BZ) + (t / (BX * BY));
  const double s = a.s;
  double vx[VPT], vy[VPT], vz[VPT];
  long long vi[VPT];
  Stencil<RC> st[VPT];
  int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
  double vmax = 0.0;
#pragma unroll
  for (int k = 0; k < VPT; ++k) {
    const int jz = jz0 + k * ZS;
    vi[k] = ((long long)jz * n + jy) * n + jx;
    vx[k] = a.vx[vi[k]];
    vy[k] = a.vy[vi[k]];
    vz[k] = a.vz[vi[k]];
    const double c = s * sqrt(vx[k] * vx[k] + vy[k] * vy[k] + vz[k] * vz[k]);
    vmax = (c >= 0.0 && vmax >= 0.0) ? fmax(vmax, c) : -1.0;  // -1: a NaN was seen
    st[k].set(jx - s * vx[k], jy - s * vy[k], jz - s * vz[k]);
    lo[0] = min(lo[0], st[k].ix);
    lo[1] = min(lo[1], st[k].iy);
    lo[2] = min(lo[2], st[k].iz);
    hi[0] = max(hi[0], st[k].ix);
    hi[1] = max(hi[1], st[k].iy);
    hi[2] = max(hi[2], st[k].iz);
  }
  block_max_cfl(vmax, cs);
  // stage 1: v at X*.  A NaN departure point gives a garbage box: the fit
  // test below then fails and the global path reads wrapped indices.
  block_box(lo, hi, red);
  int box[3], L[3];
  bool fits = box_fits(lo, hi, n, CAP, box, L);
  RC acc[VPT][8];
#pragma unroll
  for (int k = 0; k < VPT; ++k)
#pragma unroll
    for (int g = 0; g < 8; ++g) acc[k][g] = RC(0);
  const double one[4] = {1.0, 1.0, 1.0, 1.0};
  const double one1[1] = {1.0};
  if constexpr (GV == 4) {
    const double* const src[4] = {a.vx, a.vy, a.vz, nullptr};
    sl_pass<RC, 4, VPT>(tile, fits, src, one, box, L, st, n, acc, 0);
  } else {
    const double* const s2[2] = {a.vx, a.vy};
    const double* const s1[1] = {a.vz};
    const double one2[2] = {1.0, 1.0};
    sl_pass<RC, 2, VPT>(tile, fits, s2, one2, box, L, st, n, acc, 0);
    sl_pass<RC, 1, VPT>(tile, fits, s1, one1, box, L, st, n, acc, 2);
  }
  // stage 2: departure points X, then the seven fields there
  lo[0] = lo[1] = lo[2] = INT_MAX;
  hi[0] = hi[1] = hi[2] = INT_MIN;
#pragma unroll
  for (int k = 0; k < VPT; ++k) {
    const int jz = jz0 + k * ZS;
    const double Xx = jx - 0.5 * s * (vx[k] + (double)acc[k][0]);
    const double Xy = jy - 0.5 * s * (vy[k] + (double)acc[k][1]);
    const double Xz = jz - 0.5 * s * (vz[k] + (double)acc[k][2]);
    st[k].set(Xx, Xy, Xz);
    lo[0] = min(lo[0], st[k].ix);
    lo[1] = min(lo[1], st[k].iy);
    lo[2] = min(lo[2], st[k].iz);
    hi[0] = max(hi[0], st[k].ix);
    hi[1] = max(hi[1], st[k].iy);
    hi[2] = max(hi[2], st[k].iz);
#pragma unroll
    for (int g = 0; g < 8; ++g) acc[k][g] = RC(0);
  }
  block_box(lo, hi, red);
  fits = box_fits(lo, hi, n, CAP, box, L);
  double sc[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) sc[f] = sizeof(RC) == sizeof(double) ? 1.0 : pow2_scale(cs->qmax_bits[f]);
  if constexpr (GV == 4) {
    const double* const q0[4] = {a.p, a.i, a.n, a.g};
    const double* const q1[4] = {a.w, a.f, a.div, nullptr};
    const double s0[4] = {sc[0], sc[1], sc[2], sc[3]};
    const double s1[4] = {sc[4], sc[5], 1.0, 1.0};
    sl_pass<RC, 4, VPT>(tile, fits, q0, s0, box, L, st, n, acc, 0);
    sl_pass<RC, 4, VPT>(tile, fits, q1, s1, box, L, st, n, acc, 4);
  } else {
    const double* const q0[2] = {a.p, a.i};
    const double* const q1[2] = {a.n, a.g};
    const double* const q2[2] = {a.w, a.f};
    const double* const q3[1] = {a.div};
    const double s0[2] = {sc[0], sc[1]}, s1[2] = {sc[2], sc[3]}, s2[2] = {sc[4], sc[5]};
    sl_pass<RC, 2, VPT>(tile, fits, q0, s0, box, L, st, n, acc, 0);
    sl_pass<RC, 2, VPT>(tile, fits, q1, s1, box, L, st, n, acc, 2);
    sl_pass<RC, 2, VPT>(tile, fits, q2, s2, box, L, st, n, acc, 4);
    sl_pass<RC, 1, VPT>(tile, fits, q3, one1, box, L, st, n, acc, 6);
  }
  const RC dt = RC(a.dt);
  double* const outs[6] = {a.po, a.io, a.no, a.go, a.wo, a.fo};
  double unscale[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) unscale[f] = sizeof(RC) == sizeof(double) ? 1.0 : 1.0 / sc[f];
#pragma unroll
  for (int k = 0; k < VPT; ++k) {
    const RC dX = acc[k][6];
    const RC d0 = RC(a.div[vi[k]]);
    // Heun is linear in q: it runs on the scaled values, unscaled in FP64.
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      const RC qt = acc[k][f];
      const RC g0 = -qt * dX;
      const RC qs = qt + dt * g0;
      const RC gs = -qs * d0;
      outs[f][vi[k]] = (double)(qt + RC(0.5) * dt * (g0 + gs)) * unscale[f];
    }
    outs[5][vi[k]] = (double)acc[k][5] * unscale[5];
  }
}

// Bricks of 16 x 8 x 4 voxels (2 per thread) with a 2048-node (32 KiB) tile in
// both precisions: at 256^3 this measured fastest among 16x8x8, 16x16x4,
// 8x8x8 and 8x8x4 bricks with 20-64 KiB tiles (FP64 2.04 ms, FP32 2.10 ms per
// launch; an earlier per-voxel gather from node-interleaved copies took
// 6.37 + 0.67 ms and 2.29 + 0.41 ms with its packing pass).  For every
// power of two n >= 16 the bricks tile the grid, their count is a multiple of
// 8 and the bricks along z a multiple of 4, as the block-to-brick map needs.
template <typename RC>
void launch_sl_tile(const SLArgs& a, CoefScalars* cs, hipStream_t st) {
  const long long V = (long long)a.n_grid * a.n_grid * a.n_grid;
  if (sizeof(RC) != sizeof(double)) {
    const long long blocks = std::min<long long>(V / 256, 4096);
    hipLaunchKernelGGL(k_sl_scan, dim3((unsigned)blocks), dim3(256), 0, st, a, cs);
  }
  hipLaunchKernelGGL((k_sl_tile<RC, 16, 8, 4, 2048>), dim3((unsigned)(V / 512)), dim3(256), 0, st, a, cs);
}
template void launch_sl_tile<double>(const SLArgs&, CoefScalars*, hipStream_t);
template void launch_sl_tile<float>(const SLArgs&, CoefScalars*, hipStream_t);

__global__ void k_interp(int n, const double* q, const double* jx, const double* jy, const double* jz,
                         long long count, double* out) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < count;
       k += (long long)gridDim.x * blockDim.x) {
    const double* const f[1] = {q};
    double r[1];
    interp_pt<double, 1>(f, jx[k], jy[k], jz[k], n, r);
    out[k] = r[0];
  }
}

void launch_interp(int n, const double* q, const double* jx, const double* jy, const double* jz,
                   long long count, double* out, hipStream_t st) {
  if (count <= 0) return;
  long long blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_interp, dim3((unsigned)blocks), dim3(256), 0, st, n, q, jx, jy, jz, count, out);
}

// ------------------------------------------------------------ Krylov vectors
struct SpecIdx {
  int lgh, lgn, hmask, nmask, n;
  __device__ __forceinline__ void decode(long long e, int& kx, int& ky, int& kz) const {
    kx = (int)(e & hmask);
    const int iy = (int)((e >> lgh) & nmask);
    const int iz = (int)(e >> (lgh + lgn));
    ky = iy < n / 2 ? iy : (iy == n / 2 ? 0 : iy - n);
    kz = iz < n / 2 ? iz : (iz == n / 2 ? 0 : iz - n);
  }
};

static inline SpecIdx make_idx(int n) {
  int lgn = 0;
  while ((1 << lgn) < n) ++lgn;
  return SpecIdx{lgn - 1, lgn, n / 2 - 1, n - 1, n};
}

template <typename R>
__device__ __forceinline__ double wdot(cplx<R> a, cplx<R> b, int kx) {
  const double d = (double)a.x * (double)b.x + (double)a.y * (double)b.y;
  return kx == 0 ? d : 2.0 * d;
}

// r = b - ax (ax nullable); bb = ||b||^2, rr = ||r||^2 (Parseval-weighted).
template <typename R, int NC>
__global__ void __launch_bounds__(kRedThreads) k_residual(KrylovArgs a, SpecIdx ix, cplx<float>* r32) {
  const long long S = (long long)a.n * a.n * (a.n / 2);
  const cplx<R>* b = static_cast<const cplx<R>*>(a.b);
  const cplx<R>* ax = static_cast<const cplx<R>*>(a.ax);
  cplx<R>* r = static_cast<cplx<R>*>(a.r);
  double acc[2] = {0.0, 0.0};
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < S;
       e += (long long)gridDim.x * blockDim.x) {
    const int kx = (int)(e & ix.hmask);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const long long k = e + c * S;
      const cplx<R> bv = b[k];
      const cplx<R> rv = ax ? csub(bv, ax[k]) : bv;
      r[k] = rv;
      if (r32) r32[k] = {float(a.scale32 * rv.x), float(a.scale32 * rv.y)};
      acc[0] += wdot(bv, bv, kx);
      acc[1] += wdot(rv, rv, kx);
    }
  }
  block_store_partials<2>(acc, a.partials);
}

// Crank-Nicolson start: x0 = c, b = c + h Dc, r = b - (c - h Dc).
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_cn_residual(KrylovArgs a, SpecIdx ix, const cplx<R>* c,
                                                              const cplx<R>* dc) {
  const long long S = (long long)a.n * a.n * (a.n / 2);
  cplx<R>* b = static_cast<cplx<R>*>(a.b);
  cplx<R>* r = static_cast<cplx<R>*>(a.r);
  const R h = R(a.pc.h);
  double acc[2] = {0.0, 0.0};
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < S;
       e += (long long)gridDim.x * blockDim.x) {
    int kx, ky, kz;
    ix.decode(e, kx, ky, kz);
    const cplx<R> cv = c[e], dv = dc[e];
    const cplx<R> bv = {cv.x + h * dv.x, cv.y + h * dv.y};
    const cplx<R> av = {cv.x - h * dv.x, cv.y - h * dv.y};
    const cplx<R> rv = csub(bv, av);
    b[e] = bv;
    r[e] = rv;
    acc[0] += wdot(bv, bv, kx);
    acc[1] += wdot(rv, rv, kx);
  }
  block_store_partials<2>(acc, a.partials);
}

template <typename R, int NC>
__global__ void __launch_bounds__(kRedThreads) k_pcg_start(KrylovArgs a, SpecIdx ix, int zero_x) {
  const long long S = (long long)a.n * a.n * (a.n / 2);
  const cplx<R>* r = static_cast<const cplx<R>*>(a.r);
  cplx<R>* p = static_cast<cplx<R>*>(a.p);
  cplx<R>* x = static_cast<cplx<R>*>(a.x);
  double acc[1] = {0.0};
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < S;
       e += (long long)gridDim.x * blockDim.x) {
    int kx, ky, kz;
    ix.decode(e, kx, ky, kz);
    cplx<R> rv[NC], zv[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) rv[c] = r[e + c * S];
    apply_prec<R, NC>(rv, zv, kx, ky, kz, a.cs, a.pc);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      p[e + c * S] = zv[c];
      if (zero_x) x[e + c * S] = czero<R>();
      acc[0] += wdot(rv[c], zv[c], kx);
    }
  }
  block_store_partials<1>(acc, a.partials);
}

// alpha = rho / <p, q>: every block totals the inner-product pass's partials
// itself, in the order of a one-block totalling kernel, so all blocks agree;
// block 0 publishes it (or the breakdown) for the deferred x update.
__device__ __forceinline__ bool pcg_alpha(SolveScalars* sv, const double* part, int nb, int stride, double& alpha) {
  __syncthreads();  // a previous total in this block has been read (shared buffer)
  double tot[1];
  total_partials<1>(tot, part, nb, stride);
  const bool ok = isfinite(tot[0]) && tot[0] > 0.0;
  alpha = ok ? sv->rho / tot[0] : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sv->pq = tot[0];
    sv->alpha = alpha;  // 0 on breakdown: nothing left for the deferred x update to add
    if (!ok) {
      sv->bad = 1;
      sv->done = 1;
    }
  }
  return ok;
}

template <typename R, int NC>
__global__ void __launch_bounds__(kRedThreads) k_pcg_update(KrylovArgs a, SpecIdx ix) {
  if (a.sv->done) return;
  double al;
  if (!pcg_alpha(a.sv, a.dpart, a.dnb, a.dstride, al)) return;
  const long long S = (long long)a.n * a.n * (a.n / 2);
  const R alpha = R(al);
  cplx<R>* r = static_cast<cplx<R>*>(a.r);
  const cplx<R>* q = static_cast<const cplx<R>*>(a.q);
  double acc[2] = {0.0, 0.0};
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < S;
       e += (long long)gridDim.x * blockDim.x) {
    int kx, ky, kz;
    ix.decode(e, kx, ky, kz);
    cplx<R> rv[NC], zv[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const long long k = e + c * S;
      const cplx<R> qv = q[k];
      cplx<R> rr = r[k];
      rr.x -= alpha * qv.x;
      rr.y -= alpha * qv.y;
      r[k] = rr;
      rv[c] = rr;
    }
    apply_prec<R, NC>(rv, zv, kx, ky, kz, a.cs, a.pc);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      acc[0] += wdot(rv[c], rv[c], kx);
      acc[1] += wdot(rv[c], zv[c], kx);
    }
  }
  block_store_partials<2>(acc, a.partials);
}

// After an update: iteration count, ||r||^2, convergence, beta and rho.
__global__ void __launch_bounds__(kRedThreads) k_fin_update(KrylovArgs a, int nb) {
  SolveScalars* sv = a.sv;
  if (sv->done) return;
  double tot[2];
  total_partials<2>(tot, a.partials, nb, kPartialsPerBlock);
  if (threadIdx.x == 0) {
    sv->it += 1;
    sv->rr = tot[0];
    if (!(isfinite(tot[0]) && isfinite(tot[1]))) {
      sv->bad = 1;
      sv->done = 1;
    } else if (!a.fixed && tot[0] <= a.thr2) {
      sv->conv = 1;
      sv->done = 1;
    } else if (sv->it >= a.limit) {
      sv->conv = a.fixed ? 1 : 0;
      sv->done = 1;
    } else {
      sv->beta = tot[1] / sv->rho;
      sv->rho = tot[1];
    }
  }
}

// The x update of the last iteration that ran (earlier ones happen in the
// fused p-update pass of the next iteration).  Runs whatever `done` says; no
// iteration ran when it == 0.
template <typename R, int NC>
__global__ void __launch_bounds__(256) k_pcg_xfinal(KrylovArgs a) {
  if (a.sv->it == 0) return;
  const long long S = (long long)a.n * a.n * (a.n / 2);
  const R alpha = R(a.sv->alpha);
  cplx<R>* x = static_cast<cplx<R>*>(a.x);
  const cplx<R>* p = static_cast<const cplx<R>*>(a.p);
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S) return;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const cplx<R> pv = p[e + c * S];
    cplx<R> xv = x[e + c * S];
    xv.x += alpha * pv.x;
    xv.y += alpha * pv.y;
    x[e + c * S] = xv;
  }
}

template <typename R, int NC>
__global__ void __launch_bounds__(256) k_precond(KrylovArgs a, SpecIdx ix, const cplx<R>* in, cplx<R>* out) {
  const long long S = (long long)a.n * a.n * (a.n / 2);
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S) return;
  int kx, ky, kz;
  ix.decode(e, kx, ky, kz);
  cplx<R> rv[NC], zv[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) rv[c] = in[e + c * S];
  apply_prec<R, NC>(rv, zv, kx, ky, kz, a.cs, a.pc);
#pragma unroll
  for (int c = 0; c < NC; ++c) out[e + c * S] = zv[c];
}

#define TUMOR_NC_DISPATCH(nc, BODY)                    \
  if ((nc) == 1) { constexpr int NCC = 1; BODY; }      \
  else { constexpr int NCC = 3; BODY; }

static inline long long spec_count(int n) { return (long long)n * n * (n / 2); }

template <typename R>
void launch_residual(const KrylovArgs& a, void* r32, hipStream_t st) {
  const SpecIdx ix = make_idx(a.n);
  const int nb = red_blocks(spec_count(a.n));
  TUMOR_NC_DISPATCH(a.ncomp, hipLaunchKernelGGL((k_residual<R, NCC>), dim3(nb), dim3(kRedThreads), 0, st, a, ix,
                                                 static_cast<cplx<float>*>(r32)));
  hipLaunchKernelGGL(k_fin_resid, dim3(1), dim3(kRedThreads), 0, st, a.sv, a.partials, nb);
}

template <typename R>
void launch_cn_residual(const KrylovArgs& a, const void* c, const void* dc, hipStream_t st) {
  const SpecIdx ix = make_idx(a.n);
  const int nb = red_blocks(spec_count(a.n));
  hipLaunchKernelGGL((k_cn_residual<R>), dim3(nb), dim3(kRedThreads), 0, st, a, ix,
                     static_cast<const cplx<R>*>(c), static_cast<const cplx<R>*>(dc));
  hipLaunchKernelGGL(k_fin_resid, dim3(1), dim3(kRedThreads), 0, st, a.sv, a.partials, nb);
}

template <typename R>
void launch_pcg_start(const KrylovArgs& a, int zero_x, hipStream_t st) {
  const SpecIdx ix = make_idx(a.n);
  const int nb = red_blocks(spec_count(a.n));
  TUMOR_NC_DISPATCH(a.ncomp, hipLaunchKernelGGL((k_pcg_start<R, NCC>), dim3(nb), dim3(kRedThreads), 0, st, a, ix,
                                                 zero_x));
  hipLaunchKernelGGL(k_fin_start, dim3(1), dim3(kRedThreads), 0, st, a.sv, a.partials, nb);
}


template <typename R>
void launch_pcg_update(const KrylovArgs& a, hipStream_t st) {
  const SpecIdx ix = make_idx(a.n);
  const int nb = red_blocks(spec_count(a.n));
  TUMOR_NC_DISPATCH(a.ncomp, hipLaunchKernelGGL((k_pcg_update<R, NCC>), dim3(nb), dim3(kRedThreads), 0, st, a, ix));
  hipLaunchKernelGGL(k_fin_update, dim3(1), dim3(kRedThreads), 0, st, a, nb);
}

template <typename R>
void launch_pcg_xfinal(const KrylovArgs& a, hipStream_t st) {
  const long long S = spec_count(a.n);
  TUMOR_NC_DISPATCH(a.ncomp, hipLaunchKernelGGL((k_pcg_xfinal<R, NCC>), dim3((unsigned)((S + 255) / 256)),
                                                 dim3(256), 0, st, a));
}

template <typename R>
void launch_precond(const KrylovArgs& a, const void* in, void* out, hipStream_t st) {
  const SpecIdx ix = make_idx(a.n);
  const long long S = spec_count(a.n);
  TUMOR_NC_DISPATCH(a.ncomp, hipLaunchKernelGGL((k_precond<R, NCC>), dim3((unsigned)((S + 255) / 256)),
                                                 dim3(256), 0, st, a, ix, static_cast<const cplx<R>*>(in),
                                                 static_cast<cplx<R>*>(out)));
}

// ---------------------------------------------- batched independent systems
// ns one-component systems (PREC_DIFF) sharing an operator: system k's
// partials sit at slots k (and kMaxSys + k) of a block, its scalars in sv[k].
// The per-system sums run over the same elements in the same order as the
// one-system kernels, so each system's scalars equal its own solve's.
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_bresidual(BatchArgs a, SpecIdx ix, cplx<float>* r32) {
  const long long S = (long long)a.n * a.n * (a.n / 2);
  const cplx<R>* b = static_cast<const cplx<R>*>(a.b);
  const cplx<R>* ax = static_cast<const cplx<R>*>(a.ax);
  cplx<R>* r = static_cast<cplx<R>*>(a.r);
  double acc[2 * kMaxSys] = {};
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < S;
       e += (long long)gridDim.x * blockDim.x) {
    const int kx = (int)(e & ix.hmask);
#pragma unroll
    for (int c = 0; c < kMaxSys; ++c) {
      if (c >= a.ns || !(a.active & (1 << c))) continue;
      const long long k = e + c * S;
      const cplx<R> bv = b[k];
      const cplx<R> rv = ax ? csub(bv, ax[k]) : bv;
      r[k] = rv;
      if (r32) r32[k] = {float(a.scale32[c] * rv.x), float(a.scale32[c] * rv.y)};
      acc[c] += wdot(bv, bv, kx);
      acc[kMaxSys + c] += wdot(rv, rv, kx);
    }
  }
  block_store_partials<2 * kMaxSys>(acc, a.partials);
}

// Crank-Nicolson start per system: x0 = c, b = c + h Dc, r = b - (c - h Dc).
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_bcn_residual(BatchArgs a, SpecIdx ix, const cplx<R>* c,
                                                               const cplx<R>* dc) {
  const long long S = (long long)a.n * a.n * (a.n / 2);
  cplx<R>* b = static_cast<cplx<R>*>(a.b);
  cplx<R>* r = static_cast<cplx<R>*>(a.r);
  const R h = R(a.pc.h);
  double acc[2 * kMaxSys] = {};
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < S;
       e += (long long)gridDim.x * blockDim.x) {
    int kx, ky, kz;
    ix.decode(e, kx, ky, kz);
#pragma unroll
    for (int s = 0; s < kMaxSys; ++s) {
      if (s >= a.ns || !(a.active & (1 << s))) continue;
      const long long k = e + s * S;
      const cplx<R> cv = c[k], dv = dc[k];
      const cplx<R> bv = {cv.x + h * dv.x, cv.y + h * dv.y};
      const cplx<R> av = {cv.x - h * dv.x, cv.y - h * dv.y};
      const cplx<R> rv = csub(bv, av);
      b[k] = bv;
      r[k] = rv;
      acc[s] += wdot(bv, bv, kx);
      acc[kMaxSys + s] += wdot(rv, rv, kx);
    }
  }
  block_store_partials<2 * kMaxSys>(acc, a.partials);
}

__global__ void __launch_bounds__(kRedThreads) k_bfin_resid(SolveScalars* sv, int ns, int active, const double* part,
                                                             int nb) {
  double tot[2 * kMaxSys];
  total_partials<2 * kMaxSys>(tot, part, nb, kPartialsPerBlock);
  if (threadIdx.x == 0) {
    for (int s = 0; s < ns; ++s) {
      if (!(active & (1 << s))) continue;
      sv[s].bb = tot[s];
      sv[s].rr = tot[kMaxSys + s];
      sv[s].it = 0;
      sv[s].done = 0;
      sv[s].conv = 0;
      sv[s].bad = (isfinite(tot[s]) && isfinite(tot[kMaxSys + s])) ? 0 : 1;
    }
  }
}

template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_bpcg_start(BatchArgs a, SpecIdx ix, int zero_x) {
  const long long S = (long long)a.n * a.n * (a.n / 2);
  const cplx<R>* r = static_cast<const cplx<R>*>(a.r);
  cplx<R>* p = static_cast<cplx<R>*>(a.p);
  cplx<R>* x = static_cast<cplx<R>*>(a.x);
  double acc[kMaxSys] = {};
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < S;
       e += (long long)gridDim.x * blockDim.x) {
    int kx, ky, kz;
    ix.decode(e, kx, ky, kz);
#pragma unroll
    for (int s = 0; s < kMaxSys; ++s) {
      if (s >= a.ns || !(a.active & (1 << s))) continue;
      cplx<R> rv[1] = {r[e + s * S]}, zv[1];
      apply_prec<R, 1>(rv, zv, kx, ky, kz, a.cs, a.pc);
      p[e + s * S] = zv[0];
      if (zero_x) x[e + s * S] = czero<R>();
      acc[s] += wdot(rv[0], zv[0], kx);
    }
  }
  block_store_partials<kMaxSys>(acc, a.partials);
}

// rho_k = <r, M^-1 r>_k; systems outside `active` are marked done with no iterations.
__global__ void __launch_bounds__(kRedThreads) k_bfin_start(SolveScalars* sv, int ns, int active, const double* part,
                                                             int nb) {
  double tot[kMaxSys];
  total_partials<kMaxSys>(tot, part, nb, kPartialsPerBlock);
  if (threadIdx.x == 0) {
    for (int s = 0; s < ns; ++s) {
      sv[s].it = 0;
      sv[s].conv = 0;
      if (!(active & (1 << s))) {
        sv[s].done = 1;
        sv[s].bad = 0;
        continue;
      }
      sv[s].rho = tot[s];
      const bool ok = isfinite(tot[s]) && tot[s] > 0.0;
      sv[s].bad = ok ? 0 : 1;
      sv[s].done = ok ? 0 : 1;
    }
  }
}

template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_bpcg_update(BatchArgs a, SpecIdx ix) {
  const long long S = (long long)a.n * a.n * (a.n / 2);
  cplx<R>* r = static_cast<cplx<R>*>(a.r);
  const cplx<R>* q = static_cast<const cplx<R>*>(a.q);
  bool run[kMaxSys];
  R alpha[kMaxSys];
  bool any = false;
#pragma unroll
  for (int s = 0; s < kMaxSys; ++s) {
    run[s] = s < a.ns && !a.sv[s].done;  // block-uniform
    double al = 0.0;
    if (run[s]) run[s] = pcg_alpha(a.sv + s, a.dpart + s, a.dnb, kDotStride, al);
    alpha[s] = R(al);
    any = any || run[s];
  }
  if (!any) return;
  double acc[2 * kMaxSys] = {};
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < S;
       e += (long long)gridDim.x * blockDim.x) {
    int kx, ky, kz;
    ix.decode(e, kx, ky, kz);
#pragma unroll
    for (int s = 0; s < kMaxSys; ++s) {
      if (!run[s]) continue;
      const long long k = e + s * S;
      const cplx<R> qv = q[k];
      cplx<R> rr = r[k];
      rr.x -= alpha[s] * qv.x;
      rr.y -= alpha[s] * qv.y;
      r[k] = rr;
      cplx<R> rv[1] = {rr}, zv[1];
      apply_prec<R, 1>(rv, zv, kx, ky, kz, a.cs, a.pc);
      acc[s] += wdot(rv[0], rv[0], kx);
      acc[kMaxSys + s] += wdot(rv[0], zv[0], kx);
    }
  }
  block_store_partials<2 * kMaxSys>(acc, a.partials);
}

// Per system not done: iteration count, ||r||^2, convergence, beta and rho.
__global__ void __launch_bounds__(kRedThreads) k_bfin_update(BatchArgs a, int nb) {
  bool any = false;
  for (int s = 0; s < a.ns; ++s) any = any || !a.sv[s].done;
  if (!any) return;
  double tot[2 * kMaxSys];
  total_partials<2 * kMaxSys>(tot, a.partials, nb, kPartialsPerBlock);
  if (threadIdx.x == 0) {
    for (int s = 0; s < a.ns; ++s) {
      SolveScalars* sv = a.sv + s;
      if (sv->done) continue;
      const double rr = tot[s], rz = tot[kMaxSys + s];
      sv->it += 1;
      sv->rr = rr;
      if (!(isfinite(rr) && isfinite(rz))) {
        sv->bad = 1;
        sv->done = 1;
      } else if (!a.fixed[s] && rr <= a.thr2[s]) {
        sv->conv = 1;
        sv->done = 1;
      } else if (sv->it >= a.limit[s]) {
        sv->conv = a.fixed[s] ? 1 : 0;
        sv->done = 1;
      } else {
        sv->beta = rz / sv->rho;
        sv->rho = rz;
      }
    }
  }
}

// x_k += alpha_k p_k for the last iteration each system ran (none: no-op).
template <typename R>
__global__ void __launch_bounds__(256) k_bpcg_xfinal(BatchArgs a) {
  const long long S = (long long)a.n * a.n * (a.n / 2);
  cplx<R>* x = static_cast<cplx<R>*>(a.x);
  const cplx<R>* p = static_cast<const cplx<R>*>(a.p);
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S) return;
  for (int s = 0; s < a.ns; ++s) {
    if (!(a.active & (1 << s)) || a.sv[s].it == 0) continue;
    const R alpha = R(a.sv[s].alpha);
    const cplx<R> pv = p[e + s * S];
    cplx<R> xv = x[e + s * S];
    xv.x += alpha * pv.x;
    xv.y += alpha * pv.y;
    x[e + s * S] = xv;
  }
}

__global__ void k_set_flags(int* flags, int ns, int mask) {
  if ((int)threadIdx.x < ns) flags[threadIdx.x] = ((mask >> threadIdx.x) & 1) ? 0 : 1;
}

struct BScale {
  double s[kMaxSys];
};
__global__ void k_badd32to64(double* x, const float* y, BScale sc, int ns, int mask, long long count) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  for (int s = 0; s < ns; ++s)
    if (mask & (1 << s)) x[s * count + k] += sc.s[s] * (double)y[s * count + k];
}

template <typename R>
void launch_bresidual(const BatchArgs& a, void* r32, hipStream_t st) {
  const SpecIdx ix = make_idx(a.n);
  const int nb = red_blocks(spec_count(a.n));
  hipLaunchKernelGGL((k_bresidual<R>), dim3(nb), dim3(kRedThreads), 0, st, a, ix, static_cast<cplx<float>*>(r32));
  hipLaunchKernelGGL(k_bfin_resid, dim3(1), dim3(kRedThreads), 0, st, a.sv, a.ns, a.active, a.partials, nb);
}

template <typename R>
void launch_bcn_residual(const BatchArgs& a, const void* c, const void* dc, hipStream_t st) {
  const SpecIdx ix = make_idx(a.n);
  const int nb = red_blocks(spec_count(a.n));
  hipLaunchKernelGGL((k_bcn_residual<R>), dim3(nb), dim3(kRedThreads), 0, st, a, ix, static_cast<const cplx<R>*>(c),
                     static_cast<const cplx<R>*>(dc));
  hipLaunchKernelGGL(k_bfin_resid, dim3(1), dim3(kRedThreads), 0, st, a.sv, a.ns, a.active, a.partials, nb);
}

template <typename R>
void launch_bpcg_start(const BatchArgs& a, int zero_x, hipStream_t st) {
  const SpecIdx ix = make_idx(a.n);
  const int nb = red_blocks(spec_count(a.n));
  hipLaunchKernelGGL((k_bpcg_start<R>), dim3(nb), dim3(kRedThreads), 0, st, a, ix, zero_x);
  hipLaunchKernelGGL(k_bfin_start, dim3(1), dim3(kRedThreads), 0, st, a.sv, a.ns, a.active, a.partials, nb);
}


template <typename R>
void launch_bpcg_update(const BatchArgs& a, hipStream_t st) {
  const SpecIdx ix = make_idx(a.n);
  const int nb = red_blocks(spec_count(a.n));
  hipLaunchKernelGGL((k_bpcg_update<R>), dim3(nb), dim3(kRedThreads), 0, st, a, ix);
  hipLaunchKernelGGL(k_bfin_update, dim3(1), dim3(kRedThreads), 0, st, a, nb);
}

template <typename R>
void launch_bpcg_xfinal(const BatchArgs& a, hipStream_t st) {
  const long long S = spec_count(a.n);
  hipLaunchKernelGGL((k_bpcg_xfinal<R>), dim3((unsigned)((S + 255) / 256)), dim3(256), 0, st, a);
}

void launch_set_flags(int* flags, int ns, int mask, hipStream_t st) {
  hipLaunchKernelGGL(k_set_flags, dim3(1), dim3(64), 0, st, flags, ns, mask);
}

void launch_badd32to64(void* x64, const void* x32, const double (&s)[kMaxSys], int ns, int mask, long long count,
                       hipStream_t st) {
  BScale sc;
  for (int k = 0; k < kMaxSys; ++k) sc.s[k] = s[k];
  hipLaunchKernelGGL(k_badd32to64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                     static_cast<double*>(x64), static_cast<const float*>(x32), sc, ns, mask, count);
}

#define TUMOR_INST_KRYLOV(R)                                                               \
  template void launch_residual<R>(const KrylovArgs&, void*, hipStream_t);                 \
  template void launch_cn_residual<R>(const KrylovArgs&, const void*, const void*, hipStream_t); \
  template void launch_pcg_start<R>(const KrylovArgs&, int, hipStream_t);                  \
  template void launch_pcg_update<R>(const KrylovArgs&, hipStream_t);                      \
  template void launch_pcg_xfinal<R>(const KrylovArgs&, hipStream_t);                      \
  template void launch_precond<R>(const KrylovArgs&, const void*, void*, hipStream_t);     \
  template void launch_bresidual<R>(const BatchArgs&, void*, hipStream_t);                 \
  template void launch_bcn_residual<R>(const BatchArgs&, const void*, const void*, hipStream_t); \
  template void launch_bpcg_start<R>(const BatchArgs&, int, hipStream_t);                  \
  template void launch_bpcg_update<R>(const BatchArgs&, hipStream_t);                      \
  template void launch_bpcg_xfinal<R>(const BatchArgs&, hipStream_t);
TUMOR_INST_KRYLOV(double)
TUMOR_INST_KRYLOV(float)

// -------------------------------------------------------------- conversions
__global__ void k_add32to64(double* x, const float* y, double s, long long count) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) x[k] += (double)y[k] * s;
}
void launch_add32to64(void* x64, const void* x32, double s, long long count, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_add32to64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                     static_cast<double*>(x64), static_cast<const float*>(x32), s, count);
}

__global__ void k_f32_to_f64(const float* in, double* out, long long count) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) out[k] = (double)in[k];
}
void launch_f32_to_f64(const float* in, double* out, long long count, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_f32_to_f64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, in, out, count);
}

__global__ void k_scale64(double* x, double s, long long count) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) x[k] *= s;
}
void launch_scale64(double* x, double s, long long count, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_scale64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, x, s, count);
}

}  // namespace tumor
