// Moment accumulation instantiated for ARGUS_FP32.
#include "fit_accum8.h"

int fit_accum_launch_fp32(argus_ctx *ctx, const argus_fit::FitArgs &fa, int D, dim3 grid) {
    return argus_fit::fit_accum8_launch<ARGUS_FP32>(ctx, fa, D, grid);
}
