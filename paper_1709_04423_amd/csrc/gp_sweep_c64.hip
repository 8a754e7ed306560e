// complex64 instantiations of the windowed and two-pass line-sweep kernels
// (gp_sweep_kernels.h), in a translation unit of their own so that the two
// precisions compile in parallel.
#include "gp_sweep_kernels.h"

namespace gp {

hipError_t dispatch_sweep_c64(const AxisPlan &A, const SweepParams &P, gp_mode mode, int flags, bool exact,
                               bool tr, const void *tab, hipStream_t s)
{
    return mode == GP_IMAG ? dispatch_flags<float, GP_IMAG>(A, P, flags, exact, tr, tab, s)
                           : dispatch_flags<float, GP_REAL>(A, P, flags, exact, tr, tab, s);
}

}  // namespace gp
