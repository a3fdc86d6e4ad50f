// Krylov and refinement kernels, complex64 and complex128 bases
#include "krylov.inc"
#include "refine.inc"

namespace gsm {
#define GSM_KRYLOV_INST(T)                                                                  \
  template hipError_t launch_gs_dot<T>(const KrylovArgs<T>&, int, hipStream_t);            \
  template hipError_t launch_gs_update1<T>(const KrylovArgs<T>&, int, hipStream_t);        \
  template hipError_t launch_gs_update2<T>(const KrylovArgs<T>&, int, hipStream_t);        \
  template hipError_t launch_givens<T>(const KrylovArgs<T>&, int, hipStream_t);            \
  template hipError_t launch_lsq_update<T>(const KrylovArgs<T>&, hipStream_t);             \
  template hipError_t launch_cast_v0<T>(const KrylovArgs<T>&, hipStream_t);
GSM_KRYLOV_INST(float)
GSM_KRYLOV_INST(double)
}  // namespace gsm
