// The kernels of the one-workgroup-per-system engine (wg.hpp), instantiated in
// a translation unit of their own so that the library's sources compile in
// parallel.
#include "wg.hpp"

#include <hip/hip_runtime.h>

namespace mstab {
namespace wg {

template <int S>
static void launch_s(int lc, int count, Job *jobs, hipStream_t st)
{
    switch (lc) {
    case 2: hipLaunchKernelGGL((k_solve<S, 2>), dim3(count), dim3(NT), 0, st, jobs); break;
    case 4: hipLaunchKernelGGL((k_solve<S, 4>), dim3(count), dim3(NT), 0, st, jobs); break;
    default: hipLaunchKernelGGL((k_solve<S, 8>), dim3(count), dim3(NT), 0, st, jobs); break;
    }
}

void launch(int s, int lc, int count, Job *jobs, hipStream_t st)
{
    switch (s) {
    case 1: launch_s<1>(lc, count, jobs, st); break;
    case 2: launch_s<2>(lc, count, jobs, st); break;
    case 3: launch_s<3>(lc, count, jobs, st); break;
    case 4: launch_s<4>(lc, count, jobs, st); break;
    case 5: launch_s<5>(lc, count, jobs, st); break;
    case 6: launch_s<6>(lc, count, jobs, st); break;
    case 7: launch_s<7>(lc, count, jobs, st); break;
    default: launch_s<8>(lc, count, jobs, st); break;
    }
}

}  // namespace wg
}  // namespace mstab
