// instances.hip -- the objective and persistent kernel instances of one
// sample type and lane length.  Built once per pair with
//   -DPT_INST_T=<float|double> -DPT_INST_TN=<f32|f64> -DPT_INST_S=<4|8|16|32>
#define PT_INSTANCE_TU
#include "kernels.h"
#include "instances.h"

#if !defined(PT_INST_T) || !defined(PT_INST_TN) || !defined(PT_INST_S)
#error "build with -DPT_INST_T, -DPT_INST_TN and -DPT_INST_S"
#endif

#define PT_CAT3_(a, b, c) a##b##c
#define PT_CAT3(a, b, c) PT_CAT3_(a, b, c)
#define PT_NAME(stem) PT_CAT3(stem, PT_INST_TN, PT_CAT3(_s, PT_INST_S, ))

namespace pt {
namespace {

using T = PT_INST_T;
constexpr int S = PT_INST_S;

template <int C, int M>
ObjKernel pick_slope(bool slope, int lead) {
    if (lead == 2) return slope ? k_objective<T, S, C, M, true, 2> : k_objective<T, S, C, M, false, 2>;
    if (lead == 1) return slope ? k_objective<T, S, C, M, true, 1> : k_objective<T, S, C, M, false, 1>;
    return slope ? k_objective<T, S, C, M, true, 0> : k_objective<T, S, C, M, false, 0>;
}

template <int C>
ObjKernel pick_mode(int mode, bool slope, int lead) {
    if (mode == kModeMixed) return pick_slope<C, kModeMixed>(slope, lead);
    if (mode == kModePhasor) return pick_slope<C, kModePhasor>(slope, lead);
    return pick_slope<C, kModePoly>(slope, lead);
}

template <int C, int M>
PersistKernel ppick_slope(bool slope) {
    return slope ? k_fit_persistent<T, S, C, M, true> : k_fit_persistent<T, S, C, M, false>;
}

template <int C>
PersistKernel ppick_mode(int mode, bool slope) {
    if (mode == kModeMixed) return ppick_slope<C, kModeMixed>(slope);
    if (mode == kModePhasor) return ppick_slope<C, kModePhasor>(slope);
    return ppick_slope<C, kModePoly>(slope);
}

}  // namespace

ObjKernel PT_NAME(objective_kernel_)(int cpg, int mode, bool slope, int lead) {
    switch (cpg) {
        case 1: return pick_mode<1>(mode, slope, lead);
        case 2: return pick_mode<2>(mode, slope, lead);
        case 4: return pick_mode<4>(mode, slope, lead);
        default: return pick_mode<8>(mode, slope, lead);
    }
}

PersistKernel PT_NAME(persistent_kernel_)(int cpg, int mode, bool slope) {
    switch (cpg) {
        case 1: return ppick_mode<1>(mode, slope);
        case 2: return ppick_mode<2>(mode, slope);
        case 4: return ppick_mode<4>(mode, slope);
        default: return ppick_mode<8>(mode, slope);
    }
}

}  // namespace pt
