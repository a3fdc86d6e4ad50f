// plan-time kernels
#include "plan.inc"
