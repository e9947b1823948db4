// The kernels of the one-workgroup-per-system engine (wg.hpp), instantiated in
// a translation unit of their own so that the library's sources compile in
// parallel.
#include "wg.hpp"

#include <hip/hip_runtime.h>

namespace mstab {
namespace wg {

template <int S, int PM>
static void launch_s(int lc, int count, Job *jobs, hipStream_t st)
{
    switch (lc) {
    case 2: hipLaunchKernelGGL((k_solve<S, 2, PM>), dim3(count), dim3(NT), 0, st, jobs); break;
    case 4: hipLaunchKernelGGL((k_solve<S, 4, PM>), dim3(count), dim3(NT), 0, st, jobs); break;
    default: hipLaunchKernelGGL((k_solve<S, 8, PM>), dim3(count), dim3(NT), 0, st, jobs); break;
    }
}

template <int PM>
static void launch_pm(int s, int lc, int count, Job *jobs, hipStream_t st)
{
    switch (s) {
    case 1: launch_s<1, PM>(lc, count, jobs, st); break;
    case 2: launch_s<2, PM>(lc, count, jobs, st); break;
    case 3: launch_s<3, PM>(lc, count, jobs, st); break;
    case 4: launch_s<4, PM>(lc, count, jobs, st); break;
    case 5: launch_s<5, PM>(lc, count, jobs, st); break;
    case 6: launch_s<6, PM>(lc, count, jobs, st); break;
    case 7: launch_s<7, PM>(lc, count, jobs, st); break;
    default: launch_s<8, PM>(lc, count, jobs, st); break;
    }
}

void launch(int s, int lc, bool pm, int count, Job *jobs, hipStream_t st)
{
    if (pm)
        launch_pm<1>(s, lc, count, jobs, st);
    else
        launch_pm<0>(s, lc, count, jobs, st);
}

}  // namespace wg
}  // namespace mstab
