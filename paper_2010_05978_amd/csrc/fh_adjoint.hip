// fh_adjoint.hip -- vector-Jacobian products (filled in below).
#include "fh_common.hpp"
using namespace fh;
extern "C" {
fh_status fh_field_grid_vjp(fh_ctx*, const fh_quad*, double, double, int32_t, int32_t, double, double, double,
                            double, int32_t, const void*, double*, double*, double*)
{
    set_error("not implemented yet");
    return FH_ERR_UNSUPPORTED;
}
fh_status fh_starshade_vjp(fh_ctx*, int32_t, double, double, double, double, int32_t, int32_t, int32_t, int32_t,
                           const double*, int32_t, const double*, const double*, const double*, double*)
{
    set_error("not implemented yet");
    return FH_ERR_UNSUPPORTED;
}
}
