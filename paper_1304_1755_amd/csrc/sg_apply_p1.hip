// The stochastic Galerkin operator for linear elements on the triangulation
// of Sec. 6 (the kernel is in sg_apply_kernel.h).

#include "sg_apply_kernel.h"

namespace sg {

int launch_apply_p1(sg_ctx* c, const Plan& pl, const void* U, int in_float, const double* R, void* Y, int out_float,
                    int ldu, int ldy, int ldr) {
    return launch_apply_disc<true>(c, pl, U, in_float, R, Y, out_float, ldu, ldy, ldr);
}

}  // namespace sg
