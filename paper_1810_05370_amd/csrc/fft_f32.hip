// Axis-pass kernels instantiated for float arithmetic.
#include "passes_impl.hpp"

namespace tumor {
template void launch_col_pass<float>(int, int, bool, const ColProg&, const void*, hipStream_t);
template void launch_zinv_pupdate<float>(int, int, const ZPUpdateArgs&, const void*, hipStream_t);
template void launch_xinv<float>(int, const XProg&, const void*, hipStream_t);
template void launch_xfwd<float>(int, const XProg&, const void*, hipStream_t, bool);
template void launch_xelast<float>(int, const XElastArgs&, const void*, hipStream_t);
template void launch_xdiff<float>(int, const XDiffArgs&, const void*, hipStream_t);
template void launch_xforce<float>(int, const XForceArgs&, const void*, hipStream_t);
template int col_pass_blocks<float>(int, int);
}  // namespace tumor
