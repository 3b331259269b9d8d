// Deferred-launch transport kernels: the device code of karl_kernels.hip, compiled as a unit of
// their own so that they alone read the FP64 series constants from a copy in LDS (in the other
// single-job kernels the early LDS reads held too many registers).  Built, like the other
// single-job kernels, without machine-level hoisting of loop invariants.  This unit defines only
// the deferred launch and its occupancy query.
#define KARL_DRAIN_UNIT 1
#include "karl_kernels.hip"
