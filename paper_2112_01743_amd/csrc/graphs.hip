#include "internal.h"
extern "C" cpaa_status cpaa_solve_graphs(cpaa_plan_t, const double*, double, double*, cpaa_report*, void*) { return CPAA_EINVAL; }
