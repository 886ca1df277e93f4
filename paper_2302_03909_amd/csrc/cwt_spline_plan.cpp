// cwt_spline_plan.cpp -- host side of the spline method; filled in by the spline path.
#include <string>
#include "../../include/cwt.h"
#include "cwt_internal.h"
namespace cwt {
struct Wavelet;
struct TableBuilder;
[[noreturn]] void spline_unsupported();
void build_spline_plan(Plan &, const Wavelet &, TableBuilder &) { spline_unsupported(); }
}  // namespace cwt
