// 3D step kernels and launcher for one storage precision.
#include "launch3d_impl.hpp"
namespace scl {
template hipError_t launch_step3d<_Float16, float, true>(const StepArgs&, const void*, void*);
}
