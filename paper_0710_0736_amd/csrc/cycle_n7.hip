// Instantiation of the smoothing-cycle kernels for N = 7 phases.
#include "cycle_impl.hpp"

namespace acseg {
template hipError_t cycle_for_n<7>(int, int, const CycleArgs&, const CycleStep&, const CycleGrid&,
                                    CycleRole, hipStream_t);
template hipError_t step_end_for_n<7>(int, const CycleArgs&, const CycleStep&, const StepEndArgs&,
                                       const CycleArgs*, const int*, int, hipStream_t);
}  // namespace acseg
