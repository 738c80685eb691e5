// 3D step kernels and launcher for one storage precision.
#include "launch3d_impl.hpp"
namespace scl {
template hipError_t launch_step3d<float, float, false>(const StepArgs&, const void*, void*);
}
