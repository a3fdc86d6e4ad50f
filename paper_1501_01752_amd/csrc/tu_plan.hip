// plan-time kernels, the adjoint of the effective-tensor retrieval and the
// pole search
#include "plan.inc"
#include "adjoint.inc"
#include "poles.inc"
