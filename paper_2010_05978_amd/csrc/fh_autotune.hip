// fh_autotune.hip -- spread/FFT parameter search (filled in below).
#include "fh_common.hpp"
using namespace fh;
extern "C" {
fh_status fh_autotune_grid(fh_ctx*, const fh_quad*, double, double, int32_t, int32_t, double, double, const char*,
                           fh_options*)
{
    set_error("not implemented yet");
    return FH_ERR_UNSUPPORTED;
}
}
