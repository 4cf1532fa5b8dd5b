// placeholder replaced by the serving loop
#include "fv_runtime.h"
using namespace fvrt;
struct fv_server { int dummy; };
extern "C" int fv_server_create(const fv_server_desc*, fv_server** out) { if (out) *out = nullptr; return set_error(FV_E_UNSUPPORTED, "server not built"); }
extern "C" int fv_submit(fv_server*, const fv_grid_desc*, const double*, const fv_params*, double, long long, unsigned long long*) { return FV_E_UNSUPPORTED; }
extern "C" int fv_poll(fv_server*, unsigned long long, double*, size_t, fv_step_info*) { return FV_E_UNSUPPORTED; }
extern "C" int fv_cancel(fv_server*, unsigned long long) { return FV_E_UNSUPPORTED; }
extern "C" int fv_server_get_stats(fv_server*, fv_server_stats*) { return FV_E_UNSUPPORTED; }
extern "C" int fv_server_destroy(fv_server*) { return FV_E_UNSUPPORTED; }
