// Fused PT sweep (one kernel per iteration).  Not yet available: the
// runtime falls back to the unfused sweep.
#include "ep_device.h"

namespace ep {

bool fused_available(int, bool) { return false; }

template <typename R> void launch_sweep_fused_2d(const SweepArgs<R>& a, int mode, hipStream_t s)
{
    launch_sweep_unfused_2d<R>(a, mode, s);
}
template <typename R> void launch_sweep_fused_3d(const SweepArgs<R>& a, int mode, hipStream_t s)
{
    launch_sweep_unfused_3d<R>(a, mode, s);
}
template void launch_sweep_fused_2d<double>(const SweepArgs<double>&, int, hipStream_t);
template void launch_sweep_fused_2d<float>(const SweepArgs<float>&, int, hipStream_t);
template void launch_sweep_fused_3d<double>(const SweepArgs<double>&, int, hipStream_t);
template void launch_sweep_fused_3d<float>(const SweepArgs<float>&, int, hipStream_t);

}  // namespace ep
