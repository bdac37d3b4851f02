// kt_trace_w3.hip -- the trace kernels of kt_trace.hip again, in namespace
// kt_w3, built for 3 waves per SIMD.
//
// Built as kt_trace.hip is, the compiler's machine loop-invariant code motion
// lifts the FP64 constants of the polynomial series (sin/cos, asin, exp/log)
// and the stepper's coefficients out of the step loop into VGPRs, about 40
// of them; the kernel then needs ~225 VGPRs and runs 2 waves per SIMD.  This
// file is compiled with that pass off (-mllvm -disable-machine-licm, set by
// the build): each constant is then set up in scalar registers where it is
// used, a few more instructions per step, and the kernels need ~140 VGPRs,
// so 3 waves fit on a SIMD with no spills.  The third wave keeps the VALU
// busy on every issue slot, but each ray then takes longer in wall time, and
// the end of a persistent launch waits for the last rays; in this build each
// wave also cycles its priority (kt_trace.hip) so that the oldest waves do
// not take most of the issue slots.  The host picks this form when each lane
// of its grid has about four rays or more to trace (or when a launch shape
// asks for 3 or more waves per SIMD).
#define KT_TRACE_ONLY 1
#define KT_TRACE_NS kt_w3
#define KT_WAVES_PER_EU 3
#include "kt_trace.hip"
