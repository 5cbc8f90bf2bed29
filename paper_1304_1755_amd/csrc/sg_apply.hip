// The stochastic Galerkin operator for bilinear elements, and the dispatch
// over the discretisations (the kernel is in sg_apply_kernel.h); the lower
// coupling of single-partner plans.

#include "sg_apply_kernel.h"

namespace sg {

namespace {

// Lower coupling Y = R - sum_k [G_k] (x) K_k U when every output mode has at
// most one partner (the first degree level, e_k from the mean mode): one lane
// per (node, output mode) forms the one K_k u it needs from the nine values
// around its node, with no exchange between lanes and no walk.  Same
// arithmetic as k_sg_apply for such a plan (the other partner positions
// there add exact zeros).  Bilinear elements only.
template <typename Tin, typename Tout>
__global__ void __launch_bounds__(256) k_couple_one(const Tin* __restrict__ U, int ldu, const double* __restrict__ R,
                                                    int ldr, Tout* __restrict__ Y, int ldy,
                                                    const double* __restrict__ cell, const int* __restrict__ okb,
                                                    const double* __restrict__ ocoef, int n, int m, int W_out,
                                                    long total) {
    const long gl = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gl >= total) return;
    const int node = (int)(gl / W_out);
    const int t = (int)(gl - (long)node * W_out);
    const int nx = n - 1;
    const int y = node / nx, x = node - y * nx;
    const int M1 = m + 1;
    const int e = okb[t];
    const int k = e & 0xFF, b = e >> 8;
    const double g = ocoef[t];
    auto uv = [&](int xx, int yy) -> double {
        const bool in = xx >= 0 && xx < nx && yy >= 0 && yy < nx;
        const Tin v = U[((size_t)(in ? yy : 0) * nx + (in ? xx : 0)) * ldu + b];
        return in ? (double)v : 0.0;
    };
    // node (x, y); cells SW (x, y), SE (x+1, y), NW (x, y+1), NE (x+1, y+1)
    const double* cS = cell + ((size_t)y * n + x) * M1;
    const double* cN = cell + ((size_t)(y + 1) * n + x) * M1;
    const double wc = uv(x, y), wW = uv(x - 1, y), wE = uv(x + 1, y), wS = uv(x, y - 1), wN = uv(x, y + 1);
    const double wSW = uv(x - 1, y - 1), wSE = uv(x + 1, y - 1), wNW = uv(x - 1, y + 1), wNE = uv(x + 1, y + 1);
    const double uc4 = 4.0 * wc;
    const double rSW = fma(-2.0, wSW, uc4 - (wS + wW));
    const double rSE = fma(-2.0, wSE, uc4 - (wS + wE));
    const double rNW = fma(-2.0, wNW, uc4 - (wN + wW));
    const double rNE = fma(-2.0, wNE, uc4 - (wN + wE));
    const double K = fma(cS[k], rSW, fma(cS[M1 + k], rSE, fma(cN[k], rNW, cN[M1 + k] * rNE)));
    Y[(size_t)node * ldy + t] = (Tout)(R[(size_t)node * ldr + t] - fma(g, K, 0.0));
}

}  // namespace

int launch_apply(sg_ctx* c, const Plan& pl, const void* U, int in_float, const double* R, void* Y, int out_float,
                 int ldu, int ldy, int ldr) {
    if (c->hs.disc == SG_DISC_P1) return launch_apply_p1(c, pl, U, in_float, R, Y, out_float, ldu, ldy, ldr);
    const int m = c->hs.m, n = c->hs.n;
    if (pl.one_partner && R && in_float == out_float) {
        const long total = (long)c->hs.N * pl.W_out;
        if (total == 0) return SG_OK;
        const int nblk = (int)((total + 255) / 256);
        if (in_float)
            hipLaunchKernelGGL((k_couple_one<float, float>), dim3(nblk), dim3(256), 0, c->stream, (const float*)U, ldu,
                               R, ldr, (float*)Y, ldy, c->cell64, pl.d_okb, pl.d_ocoef, n, m, pl.W_out, total);
        else
            hipLaunchKernelGGL((k_couple_one<double, double>), dim3(nblk), dim3(256), 0, c->stream, (const double*)U,
                               ldu, R, ldr, (double*)Y, ldy, c->cell64, pl.d_okb, pl.d_ocoef, n, m, pl.W_out, total);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_error(std::string("coupling launch: ") + hipGetErrorString(e));
            return SG_EHIP;
        }
        return SG_OK;
    }
    return launch_apply_disc<false>(c, pl, U, in_float, R, Y, out_float, ldu, ldy, ldr);
}

}  // namespace sg
