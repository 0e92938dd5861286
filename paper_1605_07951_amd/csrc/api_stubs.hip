// Temporary: entry points not yet implemented.
#include "ctx.h"
extern "C" {
rsrr_status rsrr_basis(rsrr_ctx*, int, int, double*, int, double, double*, int, int, int*, double*) { return RSRR_EDEVICE; }
rsrr_status rsrr_project(rsrr_ctx*, const rsrr_nep*, const double*, int, int, const double*, double, double*, int, int*, rsrr_term*) { return RSRR_EDEVICE; }
rsrr_status rsrr_solve(rsrr_ctx*, const rsrr_nep*, int, const double*, int, const rsrr_term*, const double*, int, const double*, double, double, int, int, double, int, double*, double*, int, double*, int*, double*, rsrr_solve_info*) { return RSRR_EDEVICE; }
}
