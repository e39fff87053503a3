// Entry points whose GPU implementation is not built yet: they report
// ADC_ERR_UNSUPPORTED so that callers fail loudly.
#include "adc_internal.hpp"

int mlp_rank(adc_ctx, const double*, const double*, const double*, int, const std::vector<int>&, const adc_opts&,
             int r_bound) {
  return r_bound;
}
void mlp_release(adc_ctx) {}
extern "C" {
adc_status adc_stedc_batched(adc_ctx, int32_t, const int64_t*, const double* const*, const double* const*,
                             double* const*, double* const*, const int64_t*, const adc_opts*, adc_report*) {
  return ADC_ERR_UNSUPPORTED;
}
adc_status adc_mlp_features(adc_ctx, int64_t, const double*, const double*, const double*, const int64_t*,
                            int32_t, float*) {
  return ADC_ERR_UNSUPPORTED;
}
adc_status adc_mlp_init(adc_ctx, uint64_t) { return ADC_ERR_UNSUPPORTED; }
adc_status adc_mlp_train(adc_ctx, int32_t, const float*, const float*, int32_t, int32_t, float, float*) {
  return ADC_ERR_UNSUPPORTED;
}
adc_status adc_mlp_infer(adc_ctx, int32_t, const float*, float*) { return ADC_ERR_UNSUPPORTED; }
adc_status adc_mlp_grad(adc_ctx, int32_t, const float*, const float*, float*, float*) {
  return ADC_ERR_UNSUPPORTED;
}
adc_status adc_mlp_get(adc_ctx, float*) { return ADC_ERR_UNSUPPORTED; }
adc_status adc_mlp_set(adc_ctx, const float*) { return ADC_ERR_UNSUPPORTED; }
}
