// instances.h -- entry points to the objective and persistent kernel
// instances.  Every (sample type, samples per lane) pair is compiled in a
// translation unit of its own (instances.hip built once per pair), so the
// library's many template instances build in parallel; the runtime picks an
// instance through these functions.
#pragma once

#include "../../include/phasetrack.h"
#include "device.h"

namespace pt {

// k_objective(fused, nblk, total_units, lp, l_part, l_rows, l_trial, l_fpop,
// descs): the leading step's inputs first, so that kernel-argument
// preloading puts them in scalar registers (see LeadIn)
using ObjKernel = void (*)(int, int, int, int, const double*, const double*, const double*, const double*,
                           const BlockDesc*);
using PersistKernel = void (*)(const BlockDesc*, int, int, int, int, int*, uint64_t);

// Kernel arithmetic modes (template argument MODE of the kernels).
enum { kModePoly = PT_ARITH_FP64_POLY, kModeMixed = PT_ARITH_MIXED, kModePhasor = PT_ARITH_FP64_PHASOR };

// cpg: candidates per workgroup (1, 2, 4 or 8); mode: kMode*; slope: the
// amplitude-slope term is active; lead: 0 the objective alone (or with the
// last-workgroup step), 1 the leading-step instance reading the step's inputs
// from the descriptor, 2 the one taking them as kernel arguments (one block).
#define PT_DECLARE_INSTANCES(TN, S)                                                 \
    ObjKernel objective_kernel_##TN##_s##S(int cpg, int mode, bool slope, int lead); \
    PersistKernel persistent_kernel_##TN##_s##S(int cpg, int mode, bool slope);
PT_DECLARE_INSTANCES(f32, 4)
PT_DECLARE_INSTANCES(f32, 8)
PT_DECLARE_INSTANCES(f32, 16)
PT_DECLARE_INSTANCES(f32, 32)
PT_DECLARE_INSTANCES(f64, 4)
PT_DECLARE_INSTANCES(f64, 8)
PT_DECLARE_INSTANCES(f64, 16)
PT_DECLARE_INSTANCES(f64, 32)
#undef PT_DECLARE_INSTANCES

}  // namespace pt
