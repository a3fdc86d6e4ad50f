// plan-time kernels and the adjoint of the effective-tensor retrieval
#include "plan.inc"
#include "adjoint.inc"
