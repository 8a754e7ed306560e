// complex128 instantiations of the windowed and two-pass line-sweep kernels
// (gp_sweep_kernels.h), in a translation unit of their own so that the two
// precisions compile in parallel.
#include "gp_sweep_kernels.h"

namespace gp {

hipError_t dispatch_sweep_c128(const AxisPlan &A, const SweepParams &P, gp_mode mode, int flags, bool exact,
                               bool tr, const void *tab, hipStream_t s)
{
    return mode == GP_IMAG ? dispatch_flags<double, GP_IMAG>(A, P, flags, exact, tr, tab, s)
                           : dispatch_flags<double, GP_REAL>(A, P, flags, exact, tr, tab, s);
}

}  // namespace gp
