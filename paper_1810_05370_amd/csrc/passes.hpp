// Axis passes of the 3-D real FFT on the periodic N^3 grid, with the spectral
// symbols and pointwise physical-space work of each operator fused in.
//
// Layouts (all C order, x fastest):
//   physical  real    [z][y][x]                        N^3 values
//   spectral  complex [kz][ky][kxp], kxp in [0, N/2)   N^3/2 values
// The spectral array is the x-R2C half spectrum with the real Nyquist
// coefficient (kx = N/2) packed into the imaginary part of the kx = 0
// coefficient.  Both packed planes share w_x = 0 (the Nyquist wave number is
// dropped in every derivative), so every symbol used here acts on the packed
// column exactly as on the two planes separately.  Forward transforms are
// unnormalised, inverse transforms are unnormalised; the 1/N^3 lives in the
// physical-space step of each operator.
//
// Pass kinds:
//   col_pass  : FFT along y or z for a tile of TC adjacent kxp columns.  A
//               small program (ColProg) says which input columns are combined
//               with which axis symbol into each output.
//   xpass_*   : FFT along x (packed R2C / C2R) for a tile of rows, with the
//               operator's physical-space work between the inverse and the
//               forward transform, all in registers.
#pragma once
#include "fft.hpp"
#include "kernels.hpp"

namespace tumor {

constexpr int kMaxCol = 9;
constexpr int kMaxTerms = 3;

enum ColSym : int { SYM_ONE = 0, SYM_IW = 1, SYM_RAW = 2 };

struct ColTerm {
  int src;
  int sym;      // ColSym
  double coef;  // real multiplier
};

// Inverse pass: out[o] = IFFT_axis( sum_t coef_t * s_t(k) * in[src_t] )
// Forward pass: out[o] = sum_t coef_t * s_t(k) * FFT_axis(in[src_t])
//               (SYM_RAW: the input is read at the output position, untransformed)
struct ColProg {
  const void* in[kMaxCol];
  void* out[kMaxCol];
  int nout;
  int nterm[kMaxCol];
  ColTerm term[kMaxCol][kMaxTerms];
  const int* skip;  // if non-null and *skip != 0 the launch does nothing
  // per output: if non-null and *oskip[o] != 0, output o is not computed
  // (a converged system of a batched solve)
  const int* oskip[kMaxCol];
  // Optional fused Krylov inner product of a forward z pass: with dsv set,
  // each block stores its partial of sum_o <dotp[o], out[o]> (Parseval-
  // weighted) in dpart[block]; the PCG update that follows totals them
  // (col_pass_blocks blocks).  With dot_nsys > 0, output o belongs to system
  // o of a batched solve: its partial goes to dpart[block * kDotStride + o].
  const void* dotp[kMaxCol];
  SolveScalars* dsv;
  double* dpart;
  int dot_nsys;
};

// First (inverse z) pass of a Krylov operator apply with the direction update
// fused in: p = M^-1 r + beta p (in place), then out[2a] = IFFT_z(p_a) and
// out[2a+1] = IFFT_z(i w_z p_a) for the NC components.
// With nsys > 0 the vectors hold nsys independent one-component systems
// (scalars sv[0 .. nsys)); a system whose solve is done is left untouched.
struct ZPUpdateArgs {
  const void* r;
  void* p;
  void* x;  // nullable: x += alpha p with the previous p and alpha, before p is replaced
  void* out[6];
  SolveScalars* sv;
  const CoefScalars* cs;
  PrecConsts pc;
  int nsys;
};

// Rows of the x pass: generic programs.
//   xinv: phys_out[o] = scale * C2R( sum_t coef_t * s_t(kx) * in[src_t] )
//   xfwd: spec_out[o] = R2C( sum_t coef_t * phys_in[src_t] )
struct XProg {
  const void* in[kMaxCol];
  void* out[kMaxCol];
  int nout;
  int nterm[kMaxCol];
  ColTerm term[kMaxCol][kMaxTerms];
  double scale;
  const int* skip;
};

// Elasticity x pass.  Inputs (packed spectral rows, after the y and z inverse
// passes): U_x, U_y, U_z, dy u_x, dy u_y, (dz u_y + dy u_z), dz u_x, dz u_z.
// Coefficients (physical): mu, lambda, eta.  Outputs (packed spectral rows):
// eta u_x - dx s_xx, eta u_y - dx s_xy, eta u_z - dx s_xz, s_xy, s_yy, s_yz,
// s_xz, s_zz, where s = mu (grad u + grad u^T) + lambda div u I.
struct XElastArgs {
  const void* in[8];
  void* out[8];
  const void* mu;
  const void* lam;
  const void* eta;
  const int* skip;
};

// Diffusion x pass for ns fields (systems) sharing K.  Inputs per field s:
// C, dy c, dz c (packed rows) at in[3s .. 3s+2]; coefficient K.  Outputs:
// i w_x F(K dx c), F(K dy c), F(K dz c) at out[3s .. 3s+2] (each may be its
// own input).  Field s is skipped if skip[s] is non-null and *skip[s] != 0.
struct XDiffArgs {
  const void* in[9];
  void* out[9];
  const void* K;
  const int* skip[3];
  int ns;
};

// Force x pass.  Inputs: T, dy t, dz t (packed rows of tau = p + n).
// Outputs: F(-zeta tanh(tau) d_a tau), a = x, y, z.
struct XForceArgs {
  const void* in[3];
  void* out[3];
  double zeta;
};

// Products in physical space on the x pass (the coefficient sensitivities of
// the adjoint).  A factor is C2R( sum of up to kMaxTerms terms coef * s(kx) *
// in[src] ) of packed rows after the y and z inverse passes; each output is
//   out[o] (=, or += with accumulate) sum_d coef[o][d] * A_od * B_od,
// with B_od = 1 when its factor has no terms.  Outputs are physical FP64.
constexpr int kMaxDotIn = 16;
constexpr int kMaxDotOut = 6;
constexpr int kMaxDotProd = 6;
// compact term (kernel arguments are limited to 4 KiB)
struct DotTerm {
  short src;
  short sym;    // ColSym
  float coef;   // small exact multipliers (1, 2)
};
struct XFactor {
  int nterm;
  DotTerm term[kMaxTerms];
};
struct XDotArgs {
  const void* in[kMaxDotIn];
  double* out[kMaxDotOut];
  int nout;
  int accumulate[kMaxDotOut];
  int nprod[kMaxDotOut];
  XFactor fa[kMaxDotOut][kMaxDotProd];
  XFactor fb[kMaxDotOut][kMaxDotProd];
  double coef[kMaxDotOut][kMaxDotProd];
};
static_assert(sizeof(XDotArgs) <= 3072, "kernel arguments are limited to 4 KiB");

struct PassGeom {
  int n;
};

// Host-side launchers, instantiated for R = double and float.
template <typename R>
void launch_col_pass(int n, int axis /*1 = y, 2 = z*/, bool inverse, const ColProg& prog,
                     const void* tw, hipStream_t st);
template <typename R>
void launch_zinv_pupdate(int n, int ncomp, const ZPUpdateArgs& a, const void* tw, hipStream_t st);
template <typename R>
void launch_xinv(int n, const XProg& prog, const void* tw, hipStream_t st);
template <typename R>
void launch_xfwd(int n, const XProg& prog, const void* tw, hipStream_t st, bool in_fp64);
template <typename R>
void launch_xelast(int n, const XElastArgs& a, const void* tw, hipStream_t st);
template <typename R>
void launch_xdiff(int n, const XDiffArgs& a, const void* tw, hipStream_t st);
template <typename R>
void launch_xforce(int n, const XForceArgs& a, const void* tw, hipStream_t st);
template <typename R>
void launch_xdot(int n, const XDotArgs& a, const void* tw, hipStream_t st);
// blocks of a column pass along `axis` (the count of its inner-product partials)
template <typename R>
int col_pass_blocks(int n, int axis);

}  // namespace tumor
