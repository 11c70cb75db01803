// Step kernels of single lattices with x-interleaved rows (non-temporal loads and stores).
#include "ddf_step_launch.hpp"

template void ddf::host::launch_step_layout<ddf::LY_IL>(ddf_handle *, hipStream_t, int64_t);
