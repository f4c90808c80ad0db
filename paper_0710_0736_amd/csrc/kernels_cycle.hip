// kernels_cycle.hip -- launchers of the smoothing cycle and the end of a
// time step; the kernels are in cycle_impl.hpp, instantiated per phase count
// in cycle_n*.hip.
#include "cycle_impl.hpp"

namespace acseg {

int cycle_tile_rows(int N) { return cycle_ty(N); }

int cycle_launches(int sweeps) { return (sweeps + 1) / 2; }

int cycle_tiles(int N, int W, int H) {
    return ((W + kTX - 1) / kTX) * ((H + cycle_ty(N) - 1) / cycle_ty(N));
}

void cycle_tiling(int N, int W, int H, CycleArgs* a) {
    a->W = W;
    a->H = H;
    a->tiles_x = (W + kTX - 1) / kTX;
    a->tiles_y = (H + cycle_ty(N) - 1) / cycle_ty(N);
    a->ntiles = cycle_tiles(N, W, H);
    // XCD x takes tile rows [x rows_per_xcd, (x + 1) rows_per_xcd), walked in
    // strips of kStrip tile columns (workgroups per XCD: strips x kStrip x rows)
    a->rows_per_xcd = (a->tiles_y + kXcd - 1) / kXcd;
    a->tiles_per_xcd = ((a->tiles_x + kStrip - 1) / kStrip) * kStrip * a->rows_per_xcd;
}

// Convergence test after `cycles` cycles of a step (one workgroup): the
// largest per-tile residual of the last cycle against tol; marks the step done.
__global__ __launch_bounds__(kBlock) void k_step_check(CycleArgs a, int slot_idx, int cycles) {
    __shared__ float red[kBlock / kWave];
    StepSlot* slot = &a.ctl->step[slot_idx];
    if (slot->done) return;
    const float* last = a.res_part + ((cycles - 1) & 1) * a.part_stride;
    const float r = block_max(strided_max4(last, a.ntiles), red);
    if (threadIdx.x == 0 && !(r > a.tol)) {
        slot->done = 1;
        slot->cycles = cycles;
        slot->resid = r;
    }
}

hipError_t launch_step_check(const CycleArgs& a, int slot, int cycles, hipStream_t s) {
    hipLaunchKernelGGL(k_step_check, dim3(1), dim3(kBlock), 0, s, a, slot, cycles);
    return hipGetLastError();
}

hipError_t launch_cycle(int N, int C, int sweeps, const CycleArgs& a, const CycleStep& st,
                        const CycleGrid& g, CycleRole role, hipStream_t s) {
    switch (N) {
        case 2: return cycle_for_n<2>(C, sweeps, a, st, g, role, s);
        case 3: return cycle_for_n<3>(C, sweeps, a, st, g, role, s);
        case 4: return cycle_for_n<4>(C, sweeps, a, st, g, role, s);
        case 5: return cycle_for_n<5>(C, sweeps, a, st, g, role, s);
        case 6: return cycle_for_n<6>(C, sweeps, a, st, g, role, s);
        case 7: return cycle_for_n<7>(C, sweeps, a, st, g, role, s);
        case 8: return cycle_for_n<8>(C, sweeps, a, st, g, role, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_end(int N, int C, const CycleArgs& a, const CycleStep& st,
                           const StepEndArgs& e, const CycleArgs* descs, const int* imgs, int nimg,
                           hipStream_t s) {
    switch (N) {
        case 2: return step_end_for_n<2>(C, a, st, e, descs, imgs, nimg, s);
        case 3: return step_end_for_n<3>(C, a, st, e, descs, imgs, nimg, s);
        case 4: return step_end_for_n<4>(C, a, st, e, descs, imgs, nimg, s);
        case 5: return step_end_for_n<5>(C, a, st, e, descs, imgs, nimg, s);
        case 6: return step_end_for_n<6>(C, a, st, e, descs, imgs, nimg, s);
        case 7: return step_end_for_n<7>(C, a, st, e, descs, imgs, nimg, s);
        case 8: return step_end_for_n<8>(C, a, st, e, descs, imgs, nimg, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace acseg
