// rn_adjoint.hip -- reverse mode of the CG energy minimisation.
#include "rn_emin.h"

struct rn_tape {
  int placeholder;
};

extern "C" rn_status rn_tape_create(rn_ctx *ctx, rn_plan *, int32_t, int32_t, rn_tape **tape) {
  if (tape) *tape = nullptr;
  return rn_fail(ctx, RN_EINVAL, "rn_tape_create: not available in this build");
}

extern "C" void rn_tape_destroy(rn_tape *tape) { delete tape; }

rn_status rn_tape_record_begin(rn_ctx *ctx, rn_plan *, rn_tape *, int32_t, int32_t, rn_method, rn_precision) {
  return rn_fail(ctx, RN_EINVAL, "tape recording not available in this build");
}
rn_status rn_tape_record_step(rn_ctx *ctx, rn_tape *, int, const double *, const double *, int64_t, int32_t) {
  return rn_fail(ctx, RN_EINVAL, "tape recording not available in this build");
}
rn_status rn_tape_record_end(rn_ctx *ctx, rn_tape *, const double *, const int32_t *, int32_t) {
  return rn_fail(ctx, RN_EINVAL, "tape recording not available in this build");
}

extern "C" rn_status rn_energy_min_bwd(rn_ctx *ctx, rn_plan *, rn_plan *, const int32_t *, rn_tape *,
                                       const double *, const double *, double *) {
  return rn_fail(ctx, RN_EINVAL, "rn_energy_min_bwd: not available in this build");
}
