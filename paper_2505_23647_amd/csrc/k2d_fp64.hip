// 2D step kernels and launcher for one storage precision.
#include "launch2d_impl.hpp"
namespace scl {
template hipError_t launch_step2d<double, double, false>(const StepArgs&, const void*, void*, MacroRec<double>, bool);
template hipError_t launch_tile2d<double, double, false>(const StepArgs&, const void*, void*);
}
