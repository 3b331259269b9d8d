// Batched transport kernels: the device code of karl_kernels.hip, compiled as a unit of its own
// so that its build flags can differ -- the single-job kernels are built without machine-level
// hoisting of loop invariants (their hoisted FP64 constants spilled scalar registers into
// vector-register lanes), which made the batched kernel slower.  This unit defines only the
// batched launch and occupancy functions.
#define KARL_BATCHED_UNIT 1
#include "karl_kernels.hip"
