// Placeholder translation unit for the solver and the learned preconditioner.
#include "common.h"


extern "C" {
int ndl_cg_solve(const ndl_plan*, int, const double* const*, double* const*, const ndl_cg_opts*, ndl_cg_report*, void*)
{
    ndl::set_error("ndl_cg_solve not built yet");
    return NDL_EUNSUPPORTED;
}
}

extern "C" {
int ndl_net_create(int, const int*, uint64_t, ndl_net* out)
{
    if (out) *out = nullptr;
    ndl::set_error("learned preconditioner not built yet");
    return NDL_EUNSUPPORTED;
}
int ndl_net_destroy(ndl_net) { return NDL_OK; }
int ndl_net_save(ndl_net, const char*) { return NDL_EUNSUPPORTED; }
int ndl_net_load(ndl_net, const char*) { return NDL_EUNSUPPORTED; }
int ndl_net_num_params(ndl_net, int64_t*) { return NDL_EUNSUPPORTED; }
int ndl_net_train_step(ndl_net, int, int, const float*, const float*, const float*, float, float*, void*)
{
    return NDL_EUNSUPPORTED;
}
int ndl_precond_apply(ndl_net, ndl_plan, const void*, void*, void*) { return NDL_EUNSUPPORTED; }
}
