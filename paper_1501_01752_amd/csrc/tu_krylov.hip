// Krylov and refinement kernels, complex64 and complex128 bases
#include "krylov.inc"
#include "bicgstab.inc"
#include "refine.inc"

namespace gsm {
#define GSM_KRYLOV_INST(T)                                                                  \
  template hipError_t launch_cgs_dot<T>(const KrylovArgs<T>&, hipStream_t);                \
  template hipError_t launch_cgs_update<T>(const KrylovArgs<T>&, hipStream_t);             \
  template hipError_t launch_cgs_finish<T>(const KrylovArgs<T>&, hipStream_t);             \
  template hipError_t launch_lsq_update<T>(const KrylovArgs<T>&, hipStream_t);             \
  template hipError_t launch_cast_v0<T>(const KrylovArgs<T>&, hipStream_t);                 \
  template hipError_t launch_bicg<T>(const KrylovArgs<T>&, int, int, int, hipStream_t);
GSM_KRYLOV_INST(float)
GSM_KRYLOV_INST(double)
}  // namespace gsm
