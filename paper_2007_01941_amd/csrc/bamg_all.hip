// Single translation unit of the bamg library (kernels and host code).
#include "step_kernels.hip"
#include "pcg_kernels.hip"
#include "mg_plan_kernels.hip"
#include "mg_setup_kernels.hip"
#include "mg_apply_kernels.hip"
#include "adjoint_kernels.hip"
#include "layout.cpp"
#include "api.cpp"
