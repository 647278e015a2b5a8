// Spectral preconditioners of the Krylov solves, shared by the vector kernels
// and the fused FFT passes.
#pragma once
#include "kernels.hpp"

namespace tumor {

// Constant-coefficient inverses per Fourier mode (integer wave numbers
// kx, ky, kz with the Nyquist mode already mapped to 0):
//   CN diffusion:  1 / (1 + dt/2 mean(K) |w|^2)
//   elasticity:    (1/a) [I - c w w^T / (a + c |w|^2)], a = mean(eta) + mean(mu)|w|^2,
//                  c = mean(lambda) + mean(mu)  (Sherman-Morrison); a = 0 maps to 0.
template <typename R, int NC>
__device__ __forceinline__ void apply_prec(const cplx<R> (&r)[NC], cplx<R> (&z)[NC], int kx, int ky, int kz,
                                           const CoefScalars* cs, const PrecConsts& pc) {
  const double w2 = (double)kx * kx + (double)ky * ky + (double)kz * kz;
  if constexpr (NC == 1) {
    const R s = R(1.0 / (1.0 + pc.h * cs->Kbar * w2));
    z[0] = cscale(r[0], s);
  } else {
    const double a = cs->etabar + cs->mubar * w2;
    if (a > 0.0) {
      const double c = cs->lambar + cs->mubar;
      const R ia = R(1.0 / a);
      const R f = R(c / (a + c * w2));
      const R wk[3] = {R(kx), R(ky), R(kz)};
      cplx<R> wr;
      wr.x = wk[0] * r[0].x + wk[1] * r[1].x + wk[2] * r[2].x;
      wr.y = wk[0] * r[0].y + wk[1] * r[1].y + wk[2] * r[2].y;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        z[b].x = (r[b].x - f * wk[b] * wr.x) * ia;
        z[b].y = (r[b].y - f * wk[b] * wr.y) * ia;
      }
    } else {
#pragma unroll
      for (int b = 0; b < 3; ++b) z[b] = czero<R>();
    }
  }
}


}  // namespace tumor
