// FD-LBM step, fused sweep path (placeholder until the fused kernel lands).
#include "fdlbm_device.hpp"
#include "internal.hpp"

namespace fdlbm {

bool fd_sweep_supported(const FdArgs &) { return false; }

hipError_t launch_fd_sweep(const FdArgs &, int, const void *, void *, hipStream_t) { return hipErrorNotSupported; }

}  // namespace fdlbm
