// kernels_cycle.hip -- launchers of the smoothing cycle and the end of a
// time step; the kernels are in cycle_impl.hpp, instantiated per phase count
// in cycle_n*.hip.
#include "cycle_impl.hpp"

namespace acseg {

int cycle_launches(int sweeps) { return (sweeps + 1) / 2; }

int cycle_tiles(int N, int W, int H) {
    return ((W + kTX - 1) / kTX) * ((H + cycle_ty(N) - 1) / cycle_ty(N));
}

hipError_t launch_cycle(const CycleLaunch& c, hipStream_t s) {
    CycleArgs a{};
    a.bufs = c.bufs;
    a.ctl = c.ctl;
    a.image = c.image;
    a.tot = c.tot;
    a.c_prev64 = c.c_prev64;
    a.c64 = c.c64;
    a.c_out = c.c_out;
    a.rhs = c.rhs;
    a.res_part = c.res_part;
    a.cm_part = c.cm_part;
    a.part_stride = c.part_stride;
    a.coef = c.coef;
    a.rc = c.rc;
    a.tol = c.tol;
    a.slot = c.slot;
    a.cycle = c.cycle;
    a.launch = c.launch0;
    a.fixed = c.fixed ? 1 : 0;
    a.store_rhs = c.store_rhs ? 1 : 0;
    a.cm = c.cm ? 1 : 0;
    a.W = c.W;
    a.H = c.H;
    a.tiles_x = (c.W + kTX - 1) / kTX;
    a.ntiles = cycle_tiles(c.N, c.W, c.H);
    a.tiles_per_xcd = (a.ntiles + kXcd - 1) / kXcd;
    const CycleRole role{c.step_first, c.opens, c.closes};
    switch (c.N) {
        case 2: return cycle_for_n<2>(c.C, c.sweeps, a, role, s);
        case 3: return cycle_for_n<3>(c.C, c.sweeps, a, role, s);
        case 4: return cycle_for_n<4>(c.C, c.sweeps, a, role, s);
        case 5: return cycle_for_n<5>(c.C, c.sweeps, a, role, s);
        case 6: return cycle_for_n<6>(c.C, c.sweeps, a, role, s);
        case 7: return cycle_for_n<7>(c.C, c.sweeps, a, role, s);
        case 8: return cycle_for_n<8>(c.C, c.sweeps, a, role, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_end(int N, int C, int W, int H, Ctl* ctl, const float* res_part,
                           const double* cm_part, int part_stride, int max_cycles,
                           int launches_per_cycle, int slot, float tol, double* tot_next,
                           hipStream_t s) {
    StepEndArgs a{};
    a.ctl = ctl;
    a.res_part = res_part;
    a.cm_part = cm_part;
    a.tot_next = tot_next;
    a.part_stride = part_stride;
    a.ntiles = cycle_tiles(N, W, H);
    a.max_cycles = max_cycles;
    a.launches_per_cycle = launches_per_cycle;
    a.slot = slot;
    a.tol = tol;
    switch (N) {
        case 2: return step_end_for_n<2>(C, a, s);
        case 3: return step_end_for_n<3>(C, a, s);
        case 4: return step_end_for_n<4>(C, a, s);
        case 5: return step_end_for_n<5>(C, a, s);
        case 6: return step_end_for_n<6>(C, a, s);
        case 7: return step_end_for_n<7>(C, a, s);
        case 8: return step_end_for_n<8>(C, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace acseg
