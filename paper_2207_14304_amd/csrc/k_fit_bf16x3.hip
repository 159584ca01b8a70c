// Moment accumulation instantiated for ARGUS_BF16X3.
#include "fit_accum8.h"

int fit_accum_launch_bf16x3(argus_ctx *ctx, const argus_fit::FitArgs &fa, int D, dim3 grid) {
    return argus_fit::fit_accum8_launch<ARGUS_BF16X3>(ctx, fa, D, grid);
}
