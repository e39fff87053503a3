// Entry points whose GPU implementation is not built yet: they report
// ADC_ERR_UNSUPPORTED so that callers fail loudly.
#include "adc_internal.hpp"

extern "C" {
adc_status adc_stedc_batched(adc_ctx, int32_t, const int64_t*, const double* const*, const double* const*,
                             double* const*, double* const*, const int64_t*, const adc_opts*, adc_report*) {
  return ADC_ERR_UNSUPPORTED;
}

}
