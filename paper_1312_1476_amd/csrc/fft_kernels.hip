// Placeholder until the FFT kernels land: plan creation reports EUNSUPPORTED.
#include "fft.hpp"

namespace gmrf {

gmrf_status fft_plan_create(FftPlan& p, int N1, int N2) {
  (void)p; (void)N1; (void)N2;
  return GMRF_EUNSUPPORTED;
}
void fft_plan_destroy(FftPlan& p) { (void)p; }
int fft_col_blocks(const FftPlan& p) { (void)p; return 1; }

template <typename T>
void fft_apply_inv_sqrt_M(const FftPlan&, const T*, const T*, T*, T*, int, hipStream_t) {}
template <typename T>
void fft_forward_init(const FftPlan&, const double*, T*, T*, const LzState&, int, hipStream_t) {}
template <typename T>
void fft_forward_init_probes(const FftPlan&, uint64_t, const int8_t*, T*, T*, T*, const LzState&, int, hipStream_t) {}
template <typename T>
void fft_lanczos_operator(const FftPlan&, const StencilGeom&, int, const void*, const T*, const T*, T*, T*, T*,
                          const LzState&, int, int, hipStream_t) {}
template <typename T>
void fft_backward_output(const FftPlan&, const void*, const T*, double*, T*, const LzState&, int, hipStream_t) {}

#define INST(T)                                                                                            \
  template void fft_apply_inv_sqrt_M<T>(const FftPlan&, const T*, const T*, T*, T*, int, hipStream_t);     \
  template void fft_forward_init<T>(const FftPlan&, const double*, T*, T*, const LzState&, int, hipStream_t); \
  template void fft_forward_init_probes<T>(const FftPlan&, uint64_t, const int8_t*, T*, T*, T*, const LzState&, int, hipStream_t); \
  template void fft_lanczos_operator<T>(const FftPlan&, const StencilGeom&, int, const void*, const T*, const T*, T*, T*, T*, const LzState&, int, int, hipStream_t); \
  template void fft_backward_output<T>(const FftPlan&, const void*, const T*, double*, T*, const LzState&, int, hipStream_t);
INST(double)
INST(float)

}  // namespace gmrf
