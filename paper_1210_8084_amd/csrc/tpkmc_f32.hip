// FP32 instantiation of the step kernels (FMA contraction allowed; the pair
// test stays symmetric under i <-> j because every fused product negates
// exactly with its operands).
#include "tpkmc_kernels.h"

namespace tpkmc {
template void launch_key<float>(const StepArgs<float>&, hipStream_t);
template void launch_scatter<float>(const StepArgs<float>&, hipStream_t);
template void launch_prep<float>(Inst<float>*, const double*, int, int, hipStream_t);
template void launch_search<float>(const StepArgs<float>&, int, int, hipStream_t);
template void launch_search_mix<float>(const StepArgs<float>&, int, int, bool, hipStream_t);
template void launch_search_fast<float>(const StepArgs<float>&, int, hipStream_t);
template void launch_move<float>(const StepArgs<float>&, hipStream_t);
template void launch_moments<float>(const StepArgs<float>&, hipStream_t);
template void launch_random_pairs<float>(const StepArgs<float>&, hipStream_t);
template void launch_speed_stats<float>(const StepArgs<float>&, hipStream_t);
}  // namespace tpkmc
