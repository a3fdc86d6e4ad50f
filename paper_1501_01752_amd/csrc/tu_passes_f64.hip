// complex128 instantiation of the matrix-vector passes
#include "passes.inc"

namespace gsm {
template <> hipError_t launch_pass_a<double>(const PassArgs<double>& a, hipStream_t s) { return launch_pass_a_impl<double>(a, s); }
template <> hipError_t launch_pass_b<double>(const PassArgs<double>& a, hipStream_t s) { return launch_pass_b_impl<double>(a, s); }
template <> hipError_t launch_pass_c<double>(const PassArgs<double>& a, hipStream_t s) { return launch_pass_c_impl<double>(a, s); }

int pass_c_pencils_per_block(int P, bool dbl) {
  switch (P) {
#define NPB_CASE(PP) \
  case PP: return dbl ? PassCCfg<double, PP>::NPB : PassCCfg<float, PP>::NPB;
    GSM_FOR_EACH_P(NPB_CASE)
#undef NPB_CASE
    default: return 64;
  }
}
bool fft_size_supported(int P) {
  switch (P) {
#define SUP_CASE(PP) case PP: return true;
    GSM_FOR_EACH_P(SUP_CASE)
#undef SUP_CASE
    default: return false;
  }
}
}  // namespace gsm
