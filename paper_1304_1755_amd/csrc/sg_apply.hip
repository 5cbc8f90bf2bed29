// The stochastic Galerkin operator for bilinear elements, and the dispatch
// over the discretisations (the kernel is in sg_apply_kernel.h).

#include "sg_apply_kernel.h"

namespace sg {

int launch_apply(sg_ctx* c, const Plan& pl, const void* U, int in_float, const double* R, void* Y, int out_float,
                 int ldu, int ldy, int ldr) {
    if (c->hs.disc == SG_DISC_P1) return launch_apply_p1(c, pl, U, in_float, R, Y, out_float, ldu, ldy, ldr);
    return launch_apply_disc<false>(c, pl, U, in_float, R, Y, out_float, ldu, ldy, ldr);
}

}  // namespace sg
