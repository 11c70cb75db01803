// Step kernels of single lattices with row-major rows (instantiated here so that the two
// row layouts compile in parallel).
#include "ddf_step_launch.hpp"

template void ddf::host::launch_step_layout<ddf::LY_ROW>(ddf_handle *, hipStream_t, int64_t);
