// 2D step kernels and launcher for one storage precision.
#include "launch2d_impl.hpp"
namespace scl {
template hipError_t launch_step2d<float, float, true>(const StepArgs&, const void*, void*, MacroRec<float>, bool);
template hipError_t launch_tile2d<float, float, true>(const StepArgs&, const void*, void*);
}
