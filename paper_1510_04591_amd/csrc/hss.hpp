// HSS update of one DC level (Algorithms 2 and 3 on gfx950).
#pragma once
#include "adc_internal.hpp"

// Update every merge of the level whose mode is 1 (HSS): rank estimate,
// Gaussian sampling, level-by-level interpolative compression, adaptive
// check, and the HSS product U_K * H written to the merged block.  Merges
// that fail the check fall back to the dense Cauchy update.
adc_status hss_level_update(adc_ctx c, const adc_opts& o, MergeDev* h_m, MergeDev* d_m, int nm,
                            const LevelBufs& B, int depth, adc_report* rep, double* flops, double* bytes);
