// Axis-pass kernels instantiated for double arithmetic.
#include "passes_impl.hpp"

namespace tumor {
template void launch_col_pass<double>(int, int, bool, const ColProg&, const void*, hipStream_t);
template void launch_zinv_pupdate<double>(int, int, const ZPUpdateArgs&, const void*, hipStream_t);
template void launch_xinv<double>(int, const XProg&, const void*, hipStream_t);
template void launch_xfwd<double>(int, const XProg&, const void*, hipStream_t, bool);
template void launch_xelast<double>(int, const XElastArgs&, const void*, hipStream_t);
template void launch_xdiff<double>(int, const XDiffArgs&, const void*, hipStream_t);
template void launch_xforce<double>(int, const XForceArgs&, const void*, hipStream_t);
template int col_pass_blocks<double>(int, int);
template void launch_xdot<double>(int, const XDotArgs&, const void*, hipStream_t);
}  // namespace tumor
