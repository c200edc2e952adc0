// FP64 instantiation of the step kernels.  No FMA contraction: every product
// is rounded on its own, as in the CPU reference, so pair decisions and the
// post-step state agree bit for bit.
#pragma clang fp contract(off)

#include "tpkmc_kernels.h"

namespace tpkmc {
template void launch_key<double>(const StepArgs<double>&, hipStream_t);
template void launch_scatter<double>(const StepArgs<double>&, hipStream_t);
template void launch_prep<double>(Inst<double>*, const double*, int, int, hipStream_t);
template void launch_search<double>(const StepArgs<double>&, int, int, hipStream_t);
template void launch_search_mix<double>(const StepArgs<double>&, int, int, bool, hipStream_t);
template void launch_search_fast<double>(const StepArgs<double>&, int, hipStream_t);
template void launch_move<double>(const StepArgs<double>&, hipStream_t);
template void launch_moments<double>(const StepArgs<double>&, hipStream_t);
template void launch_random_pairs<double>(const StepArgs<double>&, hipStream_t);
template void launch_speed_stats<double>(const StepArgs<double>&, hipStream_t);
}  // namespace tpkmc
