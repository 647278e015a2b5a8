// Kernels and launchers of the axis passes (see passes.hpp for layouts).
#pragma once
#include <stdexcept>
#include <string>

#include "passes.hpp"
#include "prec.hpp"

namespace tumor {

// ----------------------------------------------------------------- geometry
// Column tiles: TC adjacent kxp columns, TP = N/8 threads per column.  SEG
// is the width in bytes of the contiguous segment a tile reads per position
// along the transformed axis.  Measured at 256^3: z passes, whose positions
// lie a whole plane apart, run faster with 256-byte segments; FP32 y passes
// with 128-byte segments (and twice the blocks).
template <int N, typename R, int SEG = 128>
struct ColCfg {
  static constexpr int TP = N / 8;
  static constexpr int TCW = 256 / TP;
  static constexpr int TCMIN = SEG / (2 * (int)sizeof(R));
  static constexpr int TC00 = TCW < TCMIN ? TCMIN : TCW;
  // at most 1024 threads per block, 512 in FP64 (whose passes need more
  // than the 128 VGPRs a 16-wave block leaves)
  static constexpr int MAXT = sizeof(R) == 8 ? 512 : 1024;
  static constexpr int TC0 = TC00 * TP > MAXT ? MAXT / TP : TC00;
  static constexpr int TC = (N / 2) < TC0 ? (N / 2) : TC0;
  static constexpr int THREADS = TC * TP;
  static constexpr int LDS = N * TC + N / 8 + 1;
};

// Segment width of a column pass: 256 bytes for z passes and for FP64.
template <typename R>
constexpr int col_seg(int axis) { return (axis == 2 || sizeof(R) == 8) ? 256 : 128; }

// Copy the twiddle table into LDS (all threads), so butterflies read LDS.
template <typename R, int N>
__device__ __forceinline__ void stage_twiddles(cplx<R>* stw, const cplx<R>* __restrict__ tw) {
  for (int k = threadIdx.x; k < N; k += blockDim.x) stw[k] = tw[k];
  __syncthreads();
}

// Row tiles: RW rows of L = N/2 packed complex values, TP = L/8 threads each.
template <int N>
struct RowCfg {
  static constexpr int L = N / 2;
  static constexpr int TP = L / 8;
  // One wave per block: the LDS exchanges of a row transform then wait on
  // that wave alone, and independent waves hide each other's memory latency.
  static constexpr int RW0 = 64 / TP;
  static constexpr int RW = RW0 > N * N ? N * N : RW0;
  static constexpr int THREADS = RW * TP;
  static constexpr int LP = L + L / 8;  // padded row length in LDS
};

template <int N>
__device__ __forceinline__ int xwave(int k) {  // x wave number of packed index k
  return k;                                    // k = 0 carries both kx = 0 and kx = N/2: w = 0
}

// Block sum of v stored as this block's partial of an inner product (plain
// store in slot blk, by default the workgroup's linear index; the PCG update
// that follows the pass totals the partials).
__device__ __forceinline__ double wave_sum_f(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ void store_dot_partial(double v, double* part, int stride = 1, int slot = 0, long long blk = -1) {
  __shared__ double sh[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_sum_f(v);
  __syncthreads();  // a previous call's total has read sh
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[w];
    if (blk < 0) blk = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    part[blk * stride + slot] = s;
  }
}

// ---------------------------------------------------------------- col pass
// The FP32 inner-product variant is held to 128 VGPRs (4 waves per SIMD),
// the occupancy of the other FP32 passes.
template <typename R, int N, bool INV, bool DOT, int SEG>
__global__ void __launch_bounds__((ColCfg<N, R, SEG>::THREADS), ((DOT && sizeof(R) == 4) ? 4 : 1))
    k_col_pass(ColProg prog, long long fstride, long long astride, const cplx<R>* __restrict__ twg) {
  if (prog.skip && *prog.skip) return;
  using Cfg = ColCfg<N, R, SEG>;
  constexpr int TP = Cfg::TP, TC = Cfg::TC;
  __shared__ cplx<R> sbuf[Cfg::LDS];
  __shared__ cplx<R> stw[N];
  stage_twiddles<R, N>(stw, twg);
  const cplx<R>* tw = stw;
  const int tid = threadIdx.x;
  const int col = tid % TC;
  const int t = tid / TC;
  // XCD-aware tile order of y passes.  Workgroups go round-robin to the 8
  // XCDs; the tiles are permuted so that each XCD takes whole z planes (all
  // column tiles of a plane, one after another), and its L2 and address
  // translation see an eighth of the pages.  (z passes read every plane in
  // each tile, where the order makes no difference.)
  const int gx = gridDim.x;
  const bool ypass = astride < fstride && (gridDim.y & 7u) == 0;
  const int lin = blockIdx.y * gx + blockIdx.x;
  const int bx = ypass ? (lin >> 3) % gx : (int)blockIdx.x;
  const int by = ypass ? ((lin >> 3) / gx) * 8 + (lin & 7) : (int)blockIdx.y;
  const long long blk = (long long)by * gx + bx;  // the tile's inner-product slot
  const long long base = (long long)by * fstride + (long long)bx * TC + col;
  const LdsView<R> lds{sbuf + col, TC, 1};
  double dotacc = 0.0;
  // Software pipelining: the input column of the next FFT job is loaded into
  // `nxt` before the current job's FFT, whose barriers wait on LDS only.
  auto load_col = [&](cplx<R>(&dst)[8], int src) {
    const cplx<R>* __restrict__ sp = static_cast<const cplx<R>*>(prog.in[src]);
#pragma unroll
    for (int j = 0; j < 8; ++j) dst[j] = sp[base + (long long)(t + TP * j) * astride];
  };
  // outputs to compute (block-uniform): all but those of converged systems
  unsigned am = 0;
  for (int o = 0; o < prog.nout; ++o)
    if (!(prog.oskip[o] && *prog.oskip[o])) am |= 1u << o;
  if (am == 0) return;
  // the active output after o, or -1
  auto next_out = [&](int o) -> int {
    const unsigned rest = am & ~((2u << o) - 1u);
    return rest ? __builtin_ctz(rest) : -1;
  };
  cplx<R> nxt[8];
  cplx<R> pdot[8];
  (void)pdot;
  load_col(nxt, prog.term[__builtin_ctz(am)][0].src);
  for (int o = __builtin_ctz(am); o >= 0; o = next_out(o)) {
    const int on = next_out(o);
    cplx<R> acc[8];
    const int nt = prog.nterm[o];
    if constexpr (INV) {
      {
        const ColTerm tm = prog.term[o][0];
        const R cf = R(tm.coef);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          cplx<R> v = nxt[j];
          if (tm.sym == SYM_IW) v = ciw(v, R(wavenum<N>(t + TP * j)));
          acc[j] = {cf * v.x, cf * v.y};
        }
      }
      for (int q = 1; q < nt; ++q) {
        const ColTerm tm = prog.term[o][q];
        const R cf = R(tm.coef);
        cplx<R> tmp[8];
        load_col(tmp, tm.src);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          cplx<R> v = tmp[j];
          if (tm.sym == SYM_IW) v = ciw(v, R(wavenum<N>(t + TP * j)));
          acc[j].x += cf * v.x;
          acc[j].y += cf * v.y;
        }
      }
      // nxt still holds the raw column of term 0: an output that starts from
      // the same source (and does not overwrite it) reuses it
      if (on >= 0) {
        const int ns = prog.term[on][0].src;
        if (ns != prog.term[o][0].src || prog.out[o] == prog.in[ns]) load_col(nxt, ns);
      }
      fft_block<R, N, true, 1>(acc, lds, t, tw);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = czero<R>();
      // inner-product pass: a last untransformed term read from the operand p
      // already holds p at the output positions, so it is taken after the loop
      const ColTerm last = prog.term[o][nt - 1];
      const bool rawlast = DOT && last.sym == SYM_RAW && prog.in[last.src] == prog.dotp[o];
      const int nloop = rawlast ? nt - 1 : nt;
      for (int q = 0; q < nloop; ++q) {
        const ColTerm tm = prog.term[o][q];
        const R cf = R(tm.coef);
        cplx<R> tmp[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) tmp[j] = nxt[j];
        if (q + 1 < nt) load_col(nxt, prog.term[o][q + 1].src);
        else if (on >= 0) load_col(nxt, prog.term[on][0].src);
        if (tm.sym != SYM_RAW) fft_block<R, N, false, 1>(tmp, lds, t, tw);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          cplx<R> v = tmp[j];
          if (tm.sym == SYM_IW) v = ciw(v, R(wavenum<N>(t + TP * j)));
          acc[j].x += cf * v.x;
          acc[j].y += cf * v.y;
        }
      }
      if constexpr (DOT) {
        if (rawlast) {
          const R cf = R(last.coef);
#pragma unroll
          for (int j = 0; j < 8; ++j) pdot[j] = nxt[j];
          if (on >= 0) load_col(nxt, prog.term[on][0].src);
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            acc[j].x += cf * pdot[j].x;
            acc[j].y += cf * pdot[j].y;
          }
        } else {
          // the operand loaded after the transforms: held across them it
          // would push the pass into spills
          const cplx<R>* __restrict__ pp = static_cast<const cplx<R>*>(prog.dotp[o]);
#pragma unroll
          for (int j = 0; j < 8; ++j) pdot[j] = pp[base + (long long)(t + TP * j) * astride];
        }
      }
    }
    cplx<R>* __restrict__ dst = static_cast<cplx<R>*>(prog.out[o]);
#pragma unroll
    for (int j = 0; j < 8; ++j) dst[base + (long long)(t + TP * j) * astride] = acc[j];
    if constexpr (DOT) {
#pragma unroll
      for (int j = 0; j < 8; ++j) dotacc += (double)pdot[j].x * (double)acc[j].x + (double)pdot[j].y * (double)acc[j].y;
      if (prog.dot_nsys) {
        // output o is system o's direction: its own partial
        const int kxp = bx * TC + col;
        store_dot_partial(dotacc * ((kxp == 0) ? 1.0 : 2.0), prog.dpart, kDotStride, o, blk);
        dotacc = 0.0;
      }
    }
  }
  if constexpr (DOT) {
    static_assert((N / 2 / TC) * N * kDotStride <= kPartialsCount,
                  "the inner-product partials of every block must fit the partials buffer");
    if (!prog.dot_nsys) {
      // Parseval weight: the packed kx = 0 column counts once, the others twice
      const int kxp = bx * TC + col;
      dotacc *= (kxp == 0) ? 1.0 : 2.0;
      store_dot_partial(dotacc, prog.dpart, 1, 0, blk);
    }
  }
}

template <typename R, int N, int NC>
__global__ void __launch_bounds__((ColCfg<N, R, 256>::THREADS))
    k_zinv_pupdate(ZPUpdateArgs a, const cplx<R>* __restrict__ twg) {
  if (a.sv->done) return;
  using Cfg = ColCfg<N, R, 256>;
  constexpr int TP = Cfg::TP, TC = Cfg::TC;
  constexpr long long C = N / 2;
  constexpr long long S = (long long)N * N * C;
  constexpr long long astride = (long long)N * C;
  __shared__ cplx<R> sbuf[Cfg::LDS];
  __shared__ cplx<R> stw[N];
  stage_twiddles<R, N>(stw, twg);
  const cplx<R>* tw = stw;
  const int tid = threadIdx.x;
  const int col = tid % TC;
  const int t = tid / TC;
  const int kx = blockIdx.x * TC + col;
  const int ky = wavenum<N>(blockIdx.y);
  const long long base = (long long)blockIdx.y * C + kx;
  const LdsView<R> lds{sbuf + col, TC, 1};
  const R beta = R(a.sv->beta);
  const R alpha = R(a.sv->alpha);
  const cplx<R>* __restrict__ r = static_cast<const cplx<R>*>(a.r);
  cplx<R>* __restrict__ p = static_cast<cplx<R>*>(a.p);
  cplx<R>* __restrict__ x = static_cast<cplx<R>*>(a.x);
  cplx<R> pn[NC][8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int n = t + TP * j;
    const long long idx = base + (long long)n * astride;
    cplx<R> rv[NC], zv[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) rv[c] = r[c * S + idx];
    apply_prec<R, NC>(rv, zv, kx, ky, wavenum<N>(n), a.cs, a.pc);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const cplx<R> pv = p[c * S + idx];
      if (x) {
        cplx<R> xv = x[c * S + idx];
        xv.x += alpha * pv.x;
        xv.y += alpha * pv.y;
        x[c * S + idx] = xv;
      }
      pn[c][j] = {zv[c].x + beta * pv.x, zv[c].y + beta * pv.y};
      p[c * S + idx] = pn[c][j];
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      cplx<R> acc[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = d ? ciw(pn[c][j], R(wavenum<N>(t + TP * j))) : pn[c][j];
      fft_block<R, N, true, 1>(acc, lds, t, tw);
      cplx<R>* __restrict__ dst = static_cast<cplx<R>*>(a.out[2 * c + d]);
#pragma unroll
      for (int j = 0; j < 8; ++j) dst[base + (long long)(t + TP * j) * astride] = acc[j];
    }
  }
}

// The same first pass for a.nsys independent one-component systems (a
// batched solve): blockIdx.z is the system, whose scalars are a.sv[z]; the
// blocks of a system whose solve is done exit at once.
template <typename R, int N>
__global__ void __launch_bounds__((ColCfg<N, R, 256>::THREADS))
    k_zinv_pupdate_b(ZPUpdateArgs a, const cplx<R>* __restrict__ twg) {
  const int sy = blockIdx.z;
  const SolveScalars* sv = a.sv + sy;
  if (sv->done) return;
  using Cfg = ColCfg<N, R, 256>;
  constexpr int TP = Cfg::TP, TC = Cfg::TC;
  constexpr long long C = N / 2;
  constexpr long long S = (long long)N * N * C;
  constexpr long long astride = (long long)N * C;
  __shared__ cplx<R> sbuf[Cfg::LDS];
  __shared__ cplx<R> stw[N];
  stage_twiddles<R, N>(stw, twg);
  const cplx<R>* tw = stw;
  const int tid = threadIdx.x;
  const int col = tid % TC;
  const int t = tid / TC;
  const int kx = blockIdx.x * TC + col;
  const int ky = wavenum<N>(blockIdx.y);
  const long long base = (long long)blockIdx.y * C + kx;
  const LdsView<R> lds{sbuf + col, TC, 1};
  const R beta = R(sv->beta);
  const R alpha = R(sv->alpha);
  const cplx<R>* __restrict__ r = static_cast<const cplx<R>*>(a.r);
  cplx<R>* __restrict__ p = static_cast<cplx<R>*>(a.p);
  cplx<R>* __restrict__ x = static_cast<cplx<R>*>(a.x);
  cplx<R> pn[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int n = t + TP * j;
    const long long idx = sy * S + base + (long long)n * astride;
    cplx<R> rv[1] = {r[idx]}, zv[1];
    apply_prec<R, 1>(rv, zv, kx, ky, wavenum<N>(n), a.cs, a.pc);
    const cplx<R> pv = p[idx];
    if (x) {
      cplx<R> xv = x[idx];
      xv.x += alpha * pv.x;
      xv.y += alpha * pv.y;
      x[idx] = xv;
    }
    pn[j] = {zv[0].x + beta * pv.x, zv[0].y + beta * pv.y};
    p[idx] = pn[j];
  }
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    cplx<R> acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = d ? ciw(pn[j], R(wavenum<N>(t + TP * j))) : pn[j];
    fft_block<R, N, true, 1>(acc, lds, t, tw);
    cplx<R>* __restrict__ dst = static_cast<cplx<R>*>(a.out[2 * sy + d]);
#pragma unroll
    for (int j = 0; j < 8; ++j) dst[base + (long long)(t + TP * j) * astride] = acc[j];
  }
}

// ------------------------------------------------------------- row helpers
// Pre-processing of the packed C2R: A = combined packed value at k, B at L-k.
template <typename R, int N>
__device__ __forceinline__ cplx<R> c2r_pre(cplx<R> A, cplx<R> B, int k, const cplx<R>* __restrict__ tw) {
  if (k == 0) return {A.x + A.y, A.x - A.y};
  const cplx<R> xc = cconj(B);
  const cplx<R> s = cadd(A, xc), d = csub(A, xc);
  const cplx<R> w = tw[k];
  const cplx<R> e = cmul(cconj(w), d);
  return {s.x - e.y, s.y + e.x};
}

// Packed R2C of the row held as v[j] = (x[2p], x[2p+1]), p = t + TP*j.
template <typename R, int N, bool HALF = false>
__device__ __forceinline__ void row_r2c(cplx<R> (&v)[8], const LdsRowView<R>& lds, int t,
                                        const cplx<R>* __restrict__ tw) {
  constexpr int L = N / 2, TP = L / 8;
  fft_block<R, L, false, 2, LdsRowView<R>, HALF>(v, lds, t, tw);
#pragma unroll
  for (int j = 0; j < 8; ++j) lds.put(t + TP * j, v[j]);
  __syncthreads();
  cplx<R> zc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) zc[j] = cconj(lds.get((L - (t + TP * j)) & (L - 1)));
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = t + TP * j;
    const cplx<R> z = v[j];
    if (k == 0) {
      v[j] = {z.x + z.y, z.x - z.y};
    } else {
      const cplx<R> s = cadd(z, zc[j]), d = csub(z, zc[j]);
      const cplx<R> wd = cmul(tw[k], d);
      v[j] = {R(0.5) * (s.x + wd.y), R(0.5) * (s.y - wd.x)};
    }
  }
}

// Packed C2R: gathers sum_t coef * s_t(kx) * in_t at k and L-k, pre-processes,
// inverse transforms; on return v[j] = N * (x[2p], x[2p+1]).
template <typename R, int N, bool HALF = false, typename Term>
__device__ __forceinline__ void row_c2r_terms(cplx<R> (&v)[8], int nt, const Term* terms,
                                              const void* const* in, long long rowoff,
                                              const LdsRowView<R>& lds, int t,
                                              const cplx<R>* __restrict__ tw, int off = 0) {
  constexpr int L = N / 2, TP = L / 8;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = t + TP * j;
    const int kp = (L - k) & (L - 1);
    cplx<R> A = czero<R>(), B = czero<R>();
    for (int q = 0; q < nt; ++q) {
      const Term tm = terms[q];
      const cplx<R>* __restrict__ src = static_cast<const cplx<R>*>(in[tm.src]) + rowoff;
      const R cf = R(tm.coef);
      cplx<R> a = src[off + k], b = src[off + kp];
      if (tm.sym == SYM_IW) {
        a = ciw(a, R(xwave<N>(k)));
        b = ciw(b, R(xwave<N>(kp)));
      }
      A.x += cf * a.x;
      A.y += cf * a.y;
      B.x += cf * b.x;
      B.y += cf * b.y;
    }
    v[j] = c2r_pre<R, N>(A, B, k, tw);
  }
  fft_block<R, L, true, 2, LdsRowView<R>, HALF>(v, lds, t, tw);
}

// Single-input C2R with an optional x-derivative and an optional added input.
// `off`: the row's offset from a and b (lets a block-uniform base pointer
// with a 32-bit lane offset address the row).
template <typename R, int N, bool HALF = false>
__device__ __forceinline__ void row_c2r(cplx<R> (&v)[8], const cplx<R>* __restrict__ a, bool iw_a,
                                        const cplx<R>* __restrict__ b, const LdsRowView<R>& lds, int t,
                                        const cplx<R>* __restrict__ tw, int off = 0) {
  constexpr int L = N / 2, TP = L / 8;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = t + TP * j;
    const int kp = (L - k) & (L - 1);
    cplx<R> A = a[off + k], B = a[off + kp];
    if (iw_a) {
      A = ciw(A, R(xwave<N>(k)));
      B = ciw(B, R(xwave<N>(kp)));
    }
    if (b) {
      A = cadd(A, b[off + k]);
      B = cadd(B, b[off + kp]);
    }
    v[j] = c2r_pre<R, N>(A, B, k, tw);
  }
  fft_block<R, L, true, 2, LdsRowView<R>, HALF>(v, lds, t, tw);
}

// u = C2R(U) and s = C2R(i w_x U + D) from a single read of U.
template <typename R, int N, bool HALF = false>
__device__ __forceinline__ void row_c2r_two(cplx<R> (&u)[8], cplx<R> (&s)[8], const cplx<R>* __restrict__ U,
                                            const cplx<R>* __restrict__ D, const LdsRowView<R>& lds, int t,
                                            const cplx<R>* __restrict__ tw, int off = 0) {
  constexpr int L = N / 2, TP = L / 8;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = t + TP * j;
    const int kp = (L - k) & (L - 1);
    const cplx<R> A = U[off + k], B = U[off + kp];
    u[j] = c2r_pre<R, N>(A, B, k, tw);
    s[j] = c2r_pre<R, N>(cadd(ciw(A, R(xwave<N>(k))), D[off + k]), cadd(ciw(B, R(xwave<N>(kp))), D[off + kp]), k,
                         tw);
  }
  fft_block<R, L, true, 2, LdsRowView<R>, HALF>(u, lds, t, tw);
  fft_block<R, L, true, 2, LdsRowView<R>, HALF>(s, lds, t, tw);
}

template <typename R, int N>
__device__ __forceinline__ void store_row(cplx<R>* __restrict__ dst, const cplx<R> (&v)[8], int t, int off = 0) {
  constexpr int TP = N / 16;
#pragma unroll
  for (int j = 0; j < 8; ++j) dst[off + t + TP * j] = v[j];
}

// iw_x (packed) times a row held in registers
template <typename R, int N>
__device__ __forceinline__ cplx<R> iwx(cplx<R> a, int k) {
  return ciw(a, R(xwave<N>(k)));
}

#define TUMOR_ROW_SETUP(N)                                           \
  using RC = RowCfg<N>;                                              \
  constexpr int L = RC::L, TP = RC::TP;                              \
  /* rows of a wave start 8 LDS banks apart (bank = 4 bytes, 32 banks) */ \
  constexpr int LPR = RC::LP + 32 / (int)sizeof(cplx<R>);             \
  __shared__ cplx<R> sbuf[RC::RW * LPR];                             \
  __shared__ cplx<R> stw[N];                                         \
  stage_twiddles<R, N>(stw, twg);                                    \
  const cplx<R>* tw = stw;                                           \
  const int t = threadIdx.x % TP;                                    \
  const int rl = threadIdx.x / TP;                                   \
  const long long row = row_tile() * RC::RW + rl;         \
  const LdsRowView<R> lds{sbuf + rl * LPR};                         \
  const long long soff = row * L;                                    \
  const long long poff = row * N;                                    \
  (void)soff;                                                        \
  (void)poff;

// Row tiles are taken in reverse order: the y pass before an x pass writes
// the z planes in increasing order, so the rows it wrote last, still in the
// last-level cache, are read first; and the y pass after it reads first the
// rows written last.
__device__ __forceinline__ long long row_tile() { return (long long)gridDim.x - 1 - blockIdx.x; }

// ------------------------------------------------------------- x kernels
template <typename R, int N>
__global__ void __launch_bounds__(RowCfg<N>::THREADS) k_xinv(XProg prog, const cplx<R>* __restrict__ twg) {
  if (prog.skip && *prog.skip) return;
  TUMOR_ROW_SETUP(N)
  const R scale = R(prog.scale);
  // block-uniform bases and a 32-bit lane offset, as in k_xelast
  const long long bs = row_tile() * RC::RW * L;
  const int ro = rl * L;
  for (int o = 0; o < prog.nout; ++o) {
    cplx<R> v[8];
    row_c2r_terms<R, N>(v, prog.nterm[o], prog.term[o], prog.in, bs, lds, t, tw, ro);
    cplx<R>* __restrict__ dst = static_cast<cplx<R>*>(prog.out[o]) + bs;
#pragma unroll
    for (int j = 0; j < 8; ++j) dst[ro + t + TP * j] = cscale(v[j], scale);
  }
}

template <typename R, int N, typename RIN>
__global__ void __launch_bounds__(RowCfg<N>::THREADS) k_xfwd(XProg prog, const cplx<R>* __restrict__ twg) {
  if (prog.skip && *prog.skip) return;
  TUMOR_ROW_SETUP(N)
  for (int o = 0; o < prog.nout; ++o) {
    cplx<R> v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = czero<R>();
    for (int q = 0; q < prog.nterm[o]; ++q) {
      const ColTerm tm = prog.term[o][q];
      const cplx<RIN>* __restrict__ src =
          reinterpret_cast<const cplx<RIN>*>(static_cast<const RIN*>(prog.in[tm.src]) + poff);
      const R cf = R(tm.coef);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const cplx<RIN> a = src[t + TP * j];
        v[j].x += cf * R(a.x);
        v[j].y += cf * R(a.y);
      }
    }
    row_r2c<R, N>(v, lds, t, tw);
    store_row<R, N>(static_cast<cplx<R>*>(prog.out[o]) + soff, v, t);
  }
}

template <typename R, int N>
__global__ void __launch_bounds__(RowCfg<N>::THREADS, (sizeof(R) == 4 ? 3 : 2))
    k_xelast(XElastArgs a, const cplx<R>* __restrict__ twg) {
  if (a.skip && *a.skip) return;
  constexpr bool HALF = sizeof(R) == 8;
  using RC = RowCfg<N>;
  constexpr int L = RC::L, TP = RC::TP;
  constexpr int LPR = RC::LP + 32 / (int)sizeof(cplx<R>);
  __shared__ cplx<R> sbuf[RC::RW * LPR];
  // FP64 stages half of the twiddle table (twiddle<HALF>), which leaves room
  // for the parking space at 2 waves per SIMD
  constexpr int NTW = HALF ? N / 2 : N;
  __shared__ cplx<R> stw[NTW];
  for (int k = threadIdx.x; k < NTW; k += blockDim.x) stw[k] = twg[k];
  __syncthreads();
  const cplx<R>* tw = stw;
  const int t = threadIdx.x % TP;
  const int rl = threadIdx.x / TP;
  const LdsRowView<R> lds{sbuf + rl * LPR};
  const R invV = R(1.0) / (R(N) * R(N) * R(N));
  // Rows are addressed as a block-uniform base plus a 32-bit lane offset ro
  // (the physical coefficient rows hold N reals = L complex pairs), which
  // keeps 64-bit per-lane addresses out of the registers.
  const long long bs = row_tile() * RC::RW * L;
  const int ro = rl * L;
  const cplx<R>* in[8];
#pragma unroll
  for (int f = 0; f < 8; ++f) in[f] = static_cast<const cplx<R>*>(a.in[f]) + bs;
  const cplx<R>* mu = static_cast<const cplx<R>*>(a.mu) + bs;
  const cplx<R>* lam = static_cast<const cplx<R>*>(a.lam) + bs;
  const cplx<R>* eta = static_cast<const cplx<R>*>(a.eta) + bs;
  cplx<R>* out[8];
#pragma unroll
  for (int f = 0; f < 8; ++f) out[f] = static_cast<cplx<R>*>(a.out[f]) + bs;

  // Per-thread parking space for one row (each thread reads back only its
  // own values, so no barrier is needed).
  __shared__ cplx<R> stash[RowCfg<N>::THREADS * 8];
  {
    // Group A: diagonal stresses and eta u_x.  d_x u_x, d_y u_y, d_z u_z
    // are transformed once each and the trace and the three stresses are
    // formed in one pointwise step, so mu, lambda, d_y u_y and d_z u_z are read
    // once.  One row at a time is parked in LDS, which keeps at most two rows
    // in registers.
    cplx<R> ex[8], ey[8];
    row_c2r<R, N, HALF>(ex, in[0], true, nullptr, lds, t, tw, ro);
#pragma unroll
    for (int j = 0; j < 8; ++j) stash[j * RC::THREADS + threadIdx.x] = ex[j];
    asm volatile("" ::: "memory");  // reload from LDS: ex is not kept live in registers
    row_c2r<R, N, HALF>(ey, in[4], false, nullptr, lds, t, tw, ro);
    {
      cplx<R> ez[8];
      row_c2r<R, N, HALF>(ez, in[7], false, nullptr, lds, t, tw, ro);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int p = t + TP * j;
        const cplx<R> m = mu[ro + p], l = lam[ro + p];
        ex[j] = stash[j * RC::THREADS + threadIdx.x];
        const cplx<R> ax = {ex[j].x * invV, ex[j].y * invV}, by = {ey[j].x * invV, ey[j].y * invV},
                      cz = {ez[j].x * invV, ez[j].y * invV};
        const cplx<R> lt = {l.x * (ax.x + by.x + cz.x), l.y * (ax.y + by.y + cz.y)};
        stash[j * RC::THREADS + threadIdx.x] = {R(2) * m.x * ax.x + lt.x, R(2) * m.y * ax.y + lt.y};
        ey[j] = {R(2) * m.x * by.x + lt.x, R(2) * m.y * by.y + lt.y};
        ez[j] = {R(2) * m.x * cz.x + lt.x, R(2) * m.y * cz.y + lt.y};
      }
      asm volatile("" ::: "memory");
      row_r2c<R, N, HALF>(ez, lds, t, tw);
      store_row<R, N>(out[7], ez, t, ro);
    }
    row_r2c<R, N, HALF>(ey, lds, t, tw);
    store_row<R, N>(out[4], ey, t, ro);
    // the parking space now takes mu for the three shear groups, which then
    // read it from LDS instead of global memory
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      ex[j] = stash[j * RC::THREADS + threadIdx.x];
      stash[j * RC::THREADS + threadIdx.x] = mu[ro + t + TP * j];
    }
    row_r2c<R, N, HALF>(ex, lds, t, tw);
    cplx<R> ux[8];
    row_c2r<R, N, HALF>(ux, in[0], false, nullptr, lds, t, tw, ro);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const cplx<R> e = eta[ro + t + TP * j];
      ux[j] = {e.x * ux[j].x * invV, e.y * ux[j].y * invV};
    }
    row_r2c<R, N, HALF>(ux, lds, t, tw);
#pragma unroll
    for (int j = 0; j < 8; ++j) ux[j] = csub(ux[j], iwx<R, N>(ex[j], t + TP * j));
    store_row<R, N>(out[0], ux, t, ro);
  }
  // Groups B and C: shear in the xy and xz planes with eta u_y, eta u_z.
#pragma unroll 1
  for (int g = 0; g < 2; ++g) {
    const cplx<R>* U = g == 0 ? in[1] : in[2];
    const cplx<R>* D = g == 0 ? in[3] : in[6];
    cplx<R> u[8], s[8];
    row_c2r_two<R, N, HALF>(u, s, U, D, lds, t, tw, ro);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int p = t + TP * j;
      const cplx<R> m = stash[j * RC::THREADS + threadIdx.x];
      const cplx<R> e = eta[ro + p];
      s[j] = {m.x * s[j].x * invV, m.y * s[j].y * invV};
      u[j] = {e.x * u[j].x * invV, e.y * u[j].y * invV};
    }
    row_r2c<R, N, HALF>(s, lds, t, tw);
    store_row<R, N>(g == 0 ? out[3] : out[6], s, t, ro);
    row_r2c<R, N, HALF>(u, lds, t, tw);
#pragma unroll
    for (int j = 0; j < 8; ++j) u[j] = csub(u[j], iwx<R, N>(s[j], t + TP * j));
    store_row<R, N>(g == 0 ? out[1] : out[2], u, t, ro);
  }
  // Group D: shear in the yz plane.
  {
    cplx<R> s[8];
    row_c2r<R, N, HALF>(s, in[5], false, nullptr, lds, t, tw, ro);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const cplx<R> m = stash[j * RC::THREADS + threadIdx.x];
      s[j] = {m.x * s[j].x * invV, m.y * s[j].y * invV};
    }
    row_r2c<R, N, HALF>(s, lds, t, tw);
    store_row<R, N>(out[5], s, t, ro);
  }
}

template <typename R, int N>
__global__ void __launch_bounds__(RowCfg<N>::THREADS) k_xdiff(XDiffArgs a, const cplx<R>* __restrict__ twg) {
  unsigned act = 0;  // fields to compute (block-uniform)
  for (int f = 0; f < a.ns; ++f)
    if (!(a.skip[f] && *a.skip[f])) act |= 1u << f;
  if (act == 0) return;
  TUMOR_ROW_SETUP(N)
  const R invV = R(1.0) / (R(N) * R(N) * R(N));
  // block-uniform bases and a 32-bit lane offset, as in k_xelast
  const long long bs = row_tile() * RC::RW * L;
  const int ro = rl * L;
  const cplx<R>* K = static_cast<const cplx<R>*>(a.K) + bs;
  // K / N^3 for this row, loaded once for the fields and directions
  cplx<R> kr[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const cplx<R> k = K[ro + t + TP * j];
    kr[j] = {k.x * invV, k.y * invV};
  }
#pragma unroll 1
  for (int e = 0; e < 3 * a.ns; ++e) {
    const int f = e / 3, d = e - 3 * f;
    if (!(act & (1u << f))) continue;
    // each output row is written after its own input row has been read (the
    // FFT's barriers separate them), so an output may be its input
    cplx<R> g[8];
    row_c2r<R, N>(g, static_cast<const cplx<R>*>(a.in[e]) + bs, d == 0, nullptr, lds, t, tw, ro);
#pragma unroll
    for (int j = 0; j < 8; ++j) g[j] = {kr[j].x * g[j].x, kr[j].y * g[j].y};
    row_r2c<R, N>(g, lds, t, tw);
    if (d == 0) {
#pragma unroll
      for (int j = 0; j < 8; ++j) g[j] = iwx<R, N>(g[j], t + TP * j);
    }
    store_row<R, N>(static_cast<cplx<R>*>(a.out[e]) + bs, g, t, ro);
  }
}

template <typename R>
__device__ __forceinline__ R rtanh(R x) { return tanh(x); }
template <>
__device__ __forceinline__ float rtanh<float>(float x) { return tanhf(x); }

template <typename R, int N>
__global__ void __launch_bounds__(RowCfg<N>::THREADS) k_xforce(XForceArgs a, const cplx<R>* __restrict__ twg) {
  TUMOR_ROW_SETUP(N)
  const R invV = R(1.0) / (R(N) * R(N) * R(N));
  const cplx<R>* T = static_cast<const cplx<R>*>(a.in[0]) + soff;
  cplx<R> th[8];
  row_c2r<R, N>(th, T, false, nullptr, lds, t, tw);
  const R mz = R(-a.zeta) * invV;
#pragma unroll
  for (int j = 0; j < 8; ++j) th[j] = {mz * rtanh(th[j].x * invV), mz * rtanh(th[j].y * invV)};
#pragma unroll 1
  for (int d = 0; d < 3; ++d) {
    cplx<R> g[8];
    if (d == 0) row_c2r<R, N>(g, T, true, nullptr, lds, t, tw);
    else row_c2r<R, N>(g, static_cast<const cplx<R>*>(a.in[d]) + soff, false, nullptr, lds, t, tw);
#pragma unroll
    for (int j = 0; j < 8; ++j) g[j] = {th[j].x * g[j].x, th[j].y * g[j].y};
    row_r2c<R, N>(g, lds, t, tw);
    store_row<R, N>(static_cast<cplx<R>*>(a.out[d]) + soff, g, t);
  }
}

// Sums of products of inverse-transformed rows (XDotArgs), one output at a
// time: each product's two factors are transformed in turn and multiplied
// into a running sum, so two rows and the sum are live.
template <typename R, int N>
__global__ void __launch_bounds__(RowCfg<N>::THREADS) k_xdot(XDotArgs a, const cplx<R>* __restrict__ twg) {
  TUMOR_ROW_SETUP(N)
  // block-uniform bases and a 32-bit lane offset, as in k_xelast
  const long long bs = row_tile() * RC::RW * L;
  const int ro = rl * L;
  for (int o = 0; o < a.nout; ++o) {
    cplx<R> sum[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) sum[j] = czero<R>();
    for (int d = 0; d < a.nprod[o]; ++d) {
      cplx<R> fa[8];
      row_c2r_terms<R, N>(fa, a.fa[o][d].nterm, a.fa[o][d].term, a.in, bs, lds, t, tw, ro);
      const R cf = R(a.coef[o][d]);
      if (a.fb[o][d].nterm > 0) {
        cplx<R> fb[8];
        row_c2r_terms<R, N>(fb, a.fb[o][d].nterm, a.fb[o][d].term, a.in, bs, lds, t, tw, ro);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          sum[j].x += cf * fa[j].x * fb[j].x;
          sum[j].y += cf * fa[j].y * fb[j].y;
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          sum[j].x += cf * fa[j].x;
          sum[j].y += cf * fa[j].y;
        }
      }
    }
    // physical rows hold N reals, read and written as L pairs
    cplx<R>* __restrict__ dst = reinterpret_cast<cplx<R>*>(a.out[o]) + bs;
    if (a.accumulate[o]) {
#pragma unroll
      for (int j = 0; j < 8; ++j) sum[j] = cadd(sum[j], dst[ro + t + TP * j]);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) dst[ro + t + TP * j] = sum[j];
  }
}

// ---------------------------------------------------------------- launchers
#define TUMOR_DISPATCH_N(n, ...)                                                     \
  switch (n) {                                                                       \
    case 16: { constexpr int NN = 16; __VA_ARGS__; } break;                          \
    case 32: { constexpr int NN = 32; __VA_ARGS__; } break;                          \
    case 64: { constexpr int NN = 64; __VA_ARGS__; } break;                          \
    case 128: { constexpr int NN = 128; __VA_ARGS__; } break;                        \
    case 256: { constexpr int NN = 256; __VA_ARGS__; } break;                        \
    case 512: { constexpr int NN = 512; __VA_ARGS__; } break;                        \
    default: throw std::runtime_error("unsupported grid size " + std::to_string(n)); \
  }

template <typename R, int NN, int SEG>
void launch_col_pass_seg(int axis, bool inverse, const ColProg& prog, const cplx<R>* twp, hipStream_t st) {
  using Cfg = ColCfg<NN, R, SEG>;
  const long long C = NN / 2;
  const long long fstride = axis == 1 ? (long long)NN * C : C;
  const long long astride = axis == 1 ? C : (long long)NN * C;
  dim3 grid(C / Cfg::TC, NN);
  if (inverse)
    hipLaunchKernelGGL((k_col_pass<R, NN, true, false, SEG>), grid, dim3(Cfg::THREADS), 0, st, prog, fstride,
                       astride, twp);
  else if (prog.dsv)
    hipLaunchKernelGGL((k_col_pass<R, NN, false, true, SEG>), grid, dim3(Cfg::THREADS), 0, st, prog, fstride,
                       astride, twp);
  else
    hipLaunchKernelGGL((k_col_pass<R, NN, false, false, SEG>), grid, dim3(Cfg::THREADS), 0, st, prog, fstride,
                       astride, twp);
}

template <typename R>
void launch_col_pass(int n, int axis, bool inverse, const ColProg& prog, const void* tw, hipStream_t st) {
  const cplx<R>* twp = static_cast<const cplx<R>*>(tw);
  TUMOR_DISPATCH_N(n, {
    if (col_seg<R>(axis) == 256) launch_col_pass_seg<R, NN, 256>(axis, inverse, prog, twp, st);
    else launch_col_pass_seg<R, NN, 128>(axis, inverse, prog, twp, st);
  });
}

template <typename R>
int col_pass_blocks(int n, int axis) {
  int nb = 0;
  TUMOR_DISPATCH_N(n, {
    if (col_seg<R>(axis) == 256) nb = (int)((NN / 2) / ColCfg<NN, R, 256>::TC) * NN;
    else nb = (int)((NN / 2) / ColCfg<NN, R, 128>::TC) * NN;
  });
  return nb;
}

template <typename R>
void launch_zinv_pupdate(int n, int ncomp, const ZPUpdateArgs& a, const void* tw, hipStream_t st) {
  const cplx<R>* twp = static_cast<const cplx<R>*>(tw);
  TUMOR_DISPATCH_N(n, {
    using Cfg = ColCfg<NN, R, 256>;
    dim3 grid((NN / 2) / Cfg::TC, NN);
    if (a.nsys > 0)
      hipLaunchKernelGGL((k_zinv_pupdate_b<R, NN>), dim3(grid.x, grid.y, a.nsys), dim3(Cfg::THREADS), 0, st, a, twp);
    else if (ncomp == 1)
      hipLaunchKernelGGL((k_zinv_pupdate<R, NN, 1>), grid, dim3(Cfg::THREADS), 0, st, a, twp);
    else
      hipLaunchKernelGGL((k_zinv_pupdate<R, NN, 3>), grid, dim3(Cfg::THREADS), 0, st, a, twp);
  });
}

template <typename R>
void launch_xinv(int n, const XProg& prog, const void* tw, hipStream_t st) {
  const cplx<R>* twp = static_cast<const cplx<R>*>(tw);
  TUMOR_DISPATCH_N(n, {
    dim3 grid((NN * NN) / RowCfg<NN>::RW);
    hipLaunchKernelGGL((k_xinv<R, NN>), grid, dim3(RowCfg<NN>::THREADS), 0, st, prog, twp);
  });
}

template <typename R>
void launch_xfwd(int n, const XProg& prog, const void* tw, hipStream_t st, bool in_fp64) {
  const cplx<R>* twp = static_cast<const cplx<R>*>(tw);
  TUMOR_DISPATCH_N(n, {
    dim3 grid((NN * NN) / RowCfg<NN>::RW);
    if (in_fp64)
      hipLaunchKernelGGL((k_xfwd<R, NN, double>), grid, dim3(RowCfg<NN>::THREADS), 0, st, prog, twp);
    else
      hipLaunchKernelGGL((k_xfwd<R, NN, R>), grid, dim3(RowCfg<NN>::THREADS), 0, st, prog, twp);
  });
}

template <typename R>
void launch_xelast(int n, const XElastArgs& a, const void* tw, hipStream_t st) {
  const cplx<R>* twp = static_cast<const cplx<R>*>(tw);
  TUMOR_DISPATCH_N(n, {
    dim3 grid((NN * NN) / RowCfg<NN>::RW);
    hipLaunchKernelGGL((k_xelast<R, NN>), grid, dim3(RowCfg<NN>::THREADS), 0, st, a, twp);
  });
}

template <typename R>
void launch_xdiff(int n, const XDiffArgs& a, const void* tw, hipStream_t st) {
  const cplx<R>* twp = static_cast<const cplx<R>*>(tw);
  TUMOR_DISPATCH_N(n, {
    dim3 grid((NN * NN) / RowCfg<NN>::RW);
    hipLaunchKernelGGL((k_xdiff<R, NN>), grid, dim3(RowCfg<NN>::THREADS), 0, st, a, twp);
  });
}

template <typename R>
void launch_xdot(int n, const XDotArgs& a, const void* tw, hipStream_t st) {
  static_assert(sizeof(R) == sizeof(double), "the products are formed in FP64 (physical FP64 outputs)");
  const cplx<R>* twp = static_cast<const cplx<R>*>(tw);
  TUMOR_DISPATCH_N(n, {
    dim3 grid((NN * NN) / RowCfg<NN>::RW);
    hipLaunchKernelGGL((k_xdot<R, NN>), grid, dim3(RowCfg<NN>::THREADS), 0, st, a, twp);
  });
}

template <typename R>
void launch_xforce(int n, const XForceArgs& a, const void* tw, hipStream_t st) {
  const cplx<R>* twp = static_cast<const cplx<R>*>(tw);
  TUMOR_DISPATCH_N(n, {
    dim3 grid((NN * NN) / RowCfg<NN>::RW);
    hipLaunchKernelGGL((k_xforce<R, NN>), grid, dim3(RowCfg<NN>::THREADS), 0, st, a, twp);
  });
}

}  // namespace tumor
