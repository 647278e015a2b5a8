// Batched 1-D FFT building blocks for gfx950 (CDNA4, wave64).
//
// Every transform of length L (a power of two, 8 <= L <= 512) is computed by
// TP = L/8 cooperating threads.  Thread t holds the 8 elements at positions
// t + TP*j (j = 0..7) in registers, both on input and on output (natural
// order).  Stages are Stockham autosort radix-r passes (first stage radix 8,
// later stages radix 8, 4 or 2, each thread doing 8/r butterflies), with the
// exchange between stages through LDS.  Twiddles come from a table
// tw[m] = exp(-2*pi*i*m/NT) with NT = L*TWS entries; the inverse transform
// uses conjugate twiddles and is unnormalised.
#pragma once
#include <hip/hip_runtime.h>

namespace tumor {

template <typename R>
struct __attribute__((aligned(2 * sizeof(R)))) cplx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cplx<R> cconj(cplx<R> a) { return {a.x, -a.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) { return {a.x * s, a.y * s}; }
// (i * w) * a for a real w
template <typename R>
__device__ __forceinline__ cplx<R> ciw(cplx<R> a, R w) { return {-w * a.y, w * a.x}; }
template <typename R>
__device__ __forceinline__ cplx<R> czero() { return {R(0), R(0)}; }

// Signed integer wave number with the Nyquist mode dropped (zero).
template <int N>
__device__ __forceinline__ int wavenum(int n) {
  return n < N / 2 ? n : (n == N / 2 ? 0 : n - N);
}

// ---------------------------------------------------------------- butterflies
template <typename R, bool INV>
__device__ __forceinline__ void dft2(cplx<R>* x) {
  cplx<R> a = x[0], b = x[1];
  x[0] = cadd(a, b);
  x[1] = csub(a, b);
}

template <typename R, bool INV>
__device__ __forceinline__ void dft4(cplx<R>& x0, cplx<R>& x1, cplx<R>& x2, cplx<R>& x3) {
  cplx<R> a0 = cadd(x0, x2), a1 = csub(x0, x2), a2 = cadd(x1, x3), a3 = csub(x1, x3);
  // forward: X1 = a1 - i a3, X3 = a1 + i a3 ; inverse swaps the signs
  cplx<R> ia3 = {-a3.y, a3.x};
  x0 = cadd(a0, a2);
  x2 = csub(a0, a2);
  if (INV) {
    x1 = cadd(a1, ia3);
    x3 = csub(a1, ia3);
  } else {
    x1 = csub(a1, ia3);
    x3 = cadd(a1, ia3);
  }
}

template <typename R, bool INV>
__device__ __forceinline__ void dft4(cplx<R>* x) { dft4<R, INV>(x[0], x[1], x[2], x[3]); }

template <typename R, bool INV>
__device__ __forceinline__ void dft8(cplx<R>* x) {
  const R c = R(0.70710678118654752440084436210484903928);
  cplx<R> e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
  cplx<R> o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
  dft4<R, INV>(e0, e1, e2, e3);
  dft4<R, INV>(o0, o1, o2, o3);
  // o_m *= W8^m  (forward W8 = exp(-i pi/4), inverse its conjugate)
  if (INV) {
    o1 = {c * (o1.x - o1.y), c * (o1.x + o1.y)};
    o2 = {-o2.y, o2.x};
    o3 = {-c * (o3.x + o3.y), c * (o3.x - o3.y)};
  } else {
    o1 = {c * (o1.x + o1.y), c * (o1.y - o1.x)};
    o2 = {o2.y, -o2.x};
    o3 = {c * (o3.y - o3.x), -c * (o3.x + o3.y)};
  }
  x[0] = cadd(e0, o0);
  x[4] = csub(e0, o0);
  x[1] = cadd(e1, o1);
  x[5] = csub(e1, o1);
  x[2] = cadd(e2, o2);
  x[6] = csub(e2, o2);
  x[3] = cadd(e3, o3);
  x[7] = csub(e3, o3);
}

template <typename R, bool INV, int r>
__device__ __forceinline__ void dft_r(cplx<R>* x) {
  if constexpr (r == 2) dft2<R, INV>(x);
  else if constexpr (r == 4) dft4<R, INV>(x);
  else dft8<R, INV>(x);
}

// Radix sequence per length (first stage always 8).
template <int L> struct Radix;
template <> struct Radix<8> { static constexpr int S = 1, r2 = 0, r3 = 0; };
template <> struct Radix<16> { static constexpr int S = 2, r2 = 2, r3 = 0; };
template <> struct Radix<32> { static constexpr int S = 2, r2 = 4, r3 = 0; };
template <> struct Radix<64> { static constexpr int S = 2, r2 = 8, r3 = 0; };
template <> struct Radix<128> { static constexpr int S = 3, r2 = 4, r3 = 4; };
template <> struct Radix<256> { static constexpr int S = 3, r2 = 8, r3 = 4; };
template <> struct Radix<512> { static constexpr int S = 3, r2 = 8, r3 = 8; };

// LDS view of one transform: element `pos` lives at buf[a] (a complex value,
// one 8- or 16-byte LDS access) with a = pos*ls + (pos/8)*pad (the pad breaks
// power-of-two bank strides).
template <typename R>
struct LdsView {
  cplx<R>* buf;
  int ls;
  int pad;
  __device__ __forceinline__ int addr(int pos) const { return pos * ls + (pos >> 3) * pad; }
  __device__ __forceinline__ void put(int pos, cplx<R> v) const { buf[addr(pos)] = v; }
  __device__ __forceinline__ cplx<R> get(int pos) const { return buf[addr(pos)]; }
};

// LDS view of one row transform (16 or fewer lanes per row): element `pos`
// lives at buf[pos + pos/8].  (A bijective XOR swizzle of each 16-element
// block halves the measured bank conflicts of FP32 rows but costs registers
// and no time: the row kernels wait on global memory, not on LDS.)
template <typename R>
struct LdsRowView {
  cplx<R>* buf;
  __device__ __forceinline__ int addr(int pos) const { return pos + (pos >> 3); }
  __device__ __forceinline__ void put(int pos, cplx<R> v) const { buf[addr(pos)] = v; }
  __device__ __forceinline__ cplx<R> get(int pos) const { return buf[addr(pos)]; }
};

// Twiddle m of a table of NT entries.  HALF: only the first NT/2 entries are
// stored, and entry m >= NT/2 is the negative of entry m - NT/2.
template <typename R, int NT, bool HALF>
__device__ __forceinline__ cplx<R> twiddle(const cplx<R>* __restrict__ tw, int m) {
  if constexpr (!HALF) {
    return tw[m];
  } else {
    const cplx<R> w = tw[m & (NT / 2 - 1)];
    return m < NT / 2 ? w : cplx<R>{-w.x, -w.y};
  }
}

template <typename R, int L, bool INV, int TWS, int r, int p, bool LAST, typename View, bool HALF = false>
__device__ __forceinline__ void fft_stage(cplx<R> (&v)[8], const View& lds, int t,
                                          const cplx<R>* __restrict__ tw) {
  constexpr int TP = L / 8;
  constexpr int NB = 8 / r;
  cplx<R> u[8];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int i = t + TP * b;
#pragma unroll
    for (int j = 0; j < r; ++j) u[b * r + j] = lds.get(i + j * (L / r));
  }
  if constexpr (!LAST) __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int i = t + TP * b;
    const int k = i & (p - 1);
#pragma unroll
    for (int j = 1; j < r; ++j) {
      cplx<R> w = twiddle<R, L * TWS, HALF>(tw, (j * k * (L / (p * r))) * TWS);
      if (INV) w.y = -w.y;
      u[b * r + j] = cmul(u[b * r + j], w);
    }
    dft_r<R, INV, r>(&u[b * r]);
    if constexpr (LAST) {
#pragma unroll
      for (int m = 0; m < r; ++m) v[b + m * NB] = u[b * r + m];
    } else {
#pragma unroll
      for (int m = 0; m < r; ++m) lds.put((i - k) * r + k + m * p, u[b * r + m]);
    }
  }
  if constexpr (!LAST) __syncthreads();
}

// In-place transform of the 8 register elements (positions t + TP*j).
// All threads of the block must call it (it synchronises the block).
template <typename R, int L, bool INV, int TWS, typename View, bool HALF = false>
__device__ __forceinline__ void fft_block(cplx<R> (&v)[8], const View& lds, int t,
                                          const cplx<R>* __restrict__ tw) {
  dft8<R, INV>(v);
  if constexpr (Radix<L>::S > 1) {
#pragma unroll
    for (int m = 0; m < 8; ++m) lds.put(t * 8 + m, v[m]);
    __syncthreads();
    constexpr int r2 = Radix<L>::r2;
    if constexpr (Radix<L>::S == 2) {
      fft_stage<R, L, INV, TWS, r2, 8, true, View, HALF>(v, lds, t, tw);
    } else {
      fft_stage<R, L, INV, TWS, r2, 8, false, View, HALF>(v, lds, t, tw);
      fft_stage<R, L, INV, TWS, Radix<L>::r3, 8 * r2, true, View, HALF>(v, lds, t, tw);
    }
    __syncthreads();
  }
}

}  // namespace tumor
