// complex64 instantiation of the matrix-vector passes
#include "passes.inc"

namespace gsm {
template <> hipError_t launch_pass_a<float>(const PassArgs<float>& a, hipStream_t s) { return launch_pass_a_impl<float>(a, s); }
template <> hipError_t launch_pass_b<float>(const PassArgs<float>& a, hipStream_t s) { return launch_pass_b_impl<float>(a, s); }
template <> hipError_t launch_pass_c<float>(const PassArgs<float>& a, hipStream_t s) { return launch_pass_c_impl<float>(a, s); }
}  // namespace gsm
