// fam_adjoint.hip - reverse-mode (adjoint) kernels of the FAM step.
#include <hip/hip_runtime.h>

#include "../../include/fam.h"
#include "fam_kernels.h"

struct fam_ctx;
void fam_adjoint_free(fam_ctx*) {}

extern "C" fam_status fam_adjoint(fam_ctx* ctx, const double* U0, int nsteps, double dt, int checkpoint_every,
                                  const double* dJdUT, double* dJdU0, double* J_out) {
  (void)ctx; (void)U0; (void)nsteps; (void)dt; (void)checkpoint_every; (void)dJdUT; (void)dJdU0; (void)J_out;
  return FAM_ERR_STATE;
}
