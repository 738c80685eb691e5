// 3D step kernels and launcher for one storage precision.
#include "launch3d_impl.hpp"
namespace scl {
template hipError_t launch_step3d<double, double, false>(const StepArgs&, const void*, void*);
}
