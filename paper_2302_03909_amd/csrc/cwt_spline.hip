// cwt_spline.hip -- spline method (Sec. 3.3); filled in by the spline path.
#include "cwt_internal.h"
namespace cwt {
struct TableBuilder;
hipError_t launch_spline(const Plan &, const void *, void *, void *, hipStream_t) { return hipErrorNotSupported; }
}  // namespace cwt
